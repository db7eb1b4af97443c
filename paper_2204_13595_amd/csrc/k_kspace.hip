// Long-range part: random batch Ewald (Sec. 2.2).
//   k-draw:  p vectors m_l from P_k = exp(-k^2/(4 alpha))/S, k = 2 pi m / L
//            (Eqs. (2.6)-(2.8)), per axis by inverse CDF on 64-bit Philox
//            words, the triple (0,0,0) redrawn;
//   rho:     rho_l = sum_j q_j e^{i k_l . r_j} (Eq. (2.4)) with the exact integer
//            phase (m_l . s_j) mod 2^32, FP64 accumulation, fixed-order
//            two-stage reduction;
//   force:   F_i^long,* = -ke q_i sum_l (S/p) 4 pi k_l/(V k_l^2) Im(e^{-i k_l.r_i} rho_l)
//            (Eq. (2.9)), added to the corrected short-range force and written
//            in the caller's atom order.
// Plus the adjoint (A_l = sum_m q_m (G_m . k_l) e^{i theta_ml}) and the
// energy/virial finalisation.
#include "irbe_device.hpp"
#include "irbe_internal.hpp"

namespace irbe {

// Atoms per thread and k-vectors per block row of the structure-factor kernels
// (measured optima at 3.1M atoms and p = 100: 16 atoms per thread in FP32, 8
// k-vectors per row forward and 16 in the adjoint, whose row also carries A).
template <typename real, bool ADJ>
struct RhoShape {
    static constexpr int atoms = sizeof(real) == 4 ? 16 : 8;
    static constexpr int chunk = ADJ ? 16 : 8;
};

// Blocks of the partial sums for the largest block count of any shape.
int64_t rho_blocks(int64_t n) { return blocks_for(n, kBlock * kRhoAtomsPerThread); }

// One thread per sample l: draw m_l and its FP64 constants
// kcoef[4l..4l+3] = (kx, ky, kz, c_l) with c_l = ke (S/p) 4 pi / (V k^2).
__global__ void k_ksample(int P, uint64_t seed, uint64_t step, int M, const uint64_t* __restrict__ U, double two_pi_l,
                          double coef0, int4* __restrict__ kvec, double* __restrict__ kcoef)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= P) return;
    WordStream st(seed, step, (uint32_t)l, kTagKspace);
    int m[3];
    do {
        for (int a = 0; a < 3; ++a) {
            const uint64_t hi = st.next();
            const uint64_t lo = st.next();
            const uint64_t u = (hi << 32) | lo;
            // least t in [0, 2M] with u < U[t] (U is non-decreasing, U[2M] = max)
            int a0 = 0, b0 = 2 * M;
            while (a0 < b0) {
                const int mid = (a0 + b0) >> 1;
                if (u < U[mid]) b0 = mid;
                else a0 = mid + 1;
            }
            m[a] = a0 - M;
        }
    } while (m[0] == 0 && m[1] == 0 && m[2] == 0);
    kvec[l] = make_int4(m[0], m[1], m[2], 0);
    const double kx = two_pi_l * m[0], ky = two_pi_l * m[1], kz = two_pi_l * m[2];
    const double k2 = kx * kx + ky * ky + kz * kz;
    kcoef[4 * l + 0] = kx;
    kcoef[4 * l + 1] = ky;
    kcoef[4 * l + 2] = kz;
    kcoef[4 * l + 3] = coef0 / k2;
}

hipError_t launch_ksample(irbe_ctx* h, uint64_t step)
{
    const int P = h->cfg.p_kspace;
    const double L = h->cfg.box_length;
    const double V = L * L * L;
    const double coef0 = h->cfg.coulomb_k * (h->kS / (double)P) * 4.0 * 3.14159265358979323846 / V;
    k_ksample<<<(unsigned)blocks_for(P, 64), 64, 0, h->stream>>>(P, h->cfg.seed, step, h->kM, h->ktab,
                                                                 2.0 * 3.14159265358979323846 / L, coef0, h->kvec,
                                                                 h->kcoef);
    return hipGetLastError();
}

// Partial structure factors: block (b, c) sums atoms [b*kBlock*A, ...) for the
// k-vectors of chunk c. part layout: [(l * nb + b) * NV + v], NV = 2 (rho) or
// 4 (rho and A).
template <typename real, bool ADJ>
__global__ __launch_bounds__(kBlock) void k_rho_partial(int64_t n, int P, const uint4* __restrict__ sq,
                                                        const real* __restrict__ q, const int4* __restrict__ kvec,
                                                        const double* __restrict__ kcoef, const real* __restrict__ G,
                                                        double* __restrict__ part)
{
    constexpr int A = RhoShape<real, ADJ>::atoms;
    constexpr int RC = RhoShape<real, ADJ>::chunk;
    constexpr int NV = ADJ ? 4 : 2;
    __shared__ double lds[NV * RC * (kBlock / 64)];
    const int64_t nb = gridDim.x;
    const int l0 = blockIdx.y * RC;
    uint32_t sx[A], sy[A], sz[A];
    real qa[A], gx[A], gy[A], gz[A];
#pragma unroll
    for (int a = 0; a < A; ++a) {
        const int64_t i = (int64_t)blockIdx.x * kBlock * A + (int64_t)a * kBlock + threadIdx.x;
        if (i < n) {
            const uint4 s = sq[i];
            sx[a] = s.x; sy[a] = s.y; sz[a] = s.z;
            qa[a] = q[i];
            if (ADJ) {
                gx[a] = G[3 * i]; gy[a] = G[3 * i + 1]; gz[a] = G[3 * i + 2];
            }
        } else {
            sx[a] = sy[a] = sz[a] = 0u;
            qa[a] = 0;
            gx[a] = gy[a] = gz[a] = 0;
        }
    }
    double acc[NV * RC];
#pragma unroll
    for (int c = 0; c < RC; ++c) {
        const int l = l0 + c;
        double re = 0.0, im = 0.0, are = 0.0, aim = 0.0;
        if (l < P) {
            const int4 m = kvec[l];
            real kx = 0, ky = 0, kz = 0;
            if (ADJ) {
                kx = (real)kcoef[4 * l]; ky = (real)kcoef[4 * l + 1]; kz = (real)kcoef[4 * l + 2];
            }
#pragma unroll
            for (int a = 0; a < A; ++a) {
                real sn, cs;
                Math<real>::sincos_rev(phase_rev<real>(m.x, m.y, m.z, sx[a], sy[a], sz[a]), &sn, &cs);
                re += (double)(qa[a] * cs);
                im += (double)(qa[a] * sn);
                if (ADJ) {
                    const real g = qa[a] * (gx[a] * kx + gy[a] * ky + gz[a] * kz);
                    are += (double)(g * cs);
                    aim += (double)(g * sn);
                }
            }
        }
        acc[NV * c + 0] = re;
        acc[NV * c + 1] = im;
        if (ADJ) {
            acc[NV * c + 2] = are;
            acc[NV * c + 3] = aim;
        }
    }
    double out;
    block_sum_vec<NV * RC, kBlock>(acc, lds, threadIdx.x, out);
    if (threadIdx.x < NV * RC) {
        const int c = threadIdx.x / NV, v = threadIdx.x % NV;
        const int l = l0 + c;
        if (l < P) part[((int64_t)l * nb + blockIdx.x) * NV + v] = out;
    }
}

// rho_l (and A_l) = fixed-order sums of the partials; then the per-k constants
// of the force (KForce) or adjoint (KAdj) kernels.
template <typename real, bool ADJ>
__global__ __launch_bounds__(kReduceBlock) void k_rho_final(int64_t nb, const double* __restrict__ part,
                                                            const double* __restrict__ kcoef, double* __restrict__ rho,
                                                            double* __restrict__ Avec, void* __restrict__ kconst)
{
    constexpr int NV = ADJ ? 4 : 2;
    __shared__ double lds[NV * (kReduceBlock / 64)];
    const int l = blockIdx.x;
    double vals[NV];
    for (int v = 0; v < NV; ++v) vals[v] = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += kReduceBlock)
        for (int v = 0; v < NV; ++v) vals[v] += part[((int64_t)l * nb + b) * NV + v];
    double out;
    block_sum_vec<NV, kReduceBlock>(vals, lds, threadIdx.x, out);
    __shared__ double tot[4];
    if (threadIdx.x < NV) tot[threadIdx.x] = out;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double c = kcoef[4 * l + 3];
        rho[2 * l] = tot[0];
        rho[2 * l + 1] = tot[1];
        if (!ADJ) {
            KForce<real> kf;
            kf.kx = (real)kcoef[4 * l];
            kf.ky = (real)kcoef[4 * l + 1];
            kf.kz = (real)kcoef[4 * l + 2];
            kf.a = (real)(c * tot[1]);
            kf.b = (real)(c * tot[0]);
            kf.pad0 = kf.pad1 = kf.pad2 = 0;
            ((KForce<real>*)kconst)[l] = kf;
        } else {
            Avec[2 * l] = tot[2];
            Avec[2 * l + 1] = tot[3];
            KAdj<real> ka;
            ka.kx = (real)kcoef[4 * l];
            ka.ky = (real)kcoef[4 * l + 1];
            ka.kz = (real)kcoef[4 * l + 2];
            ka.ar = (real)(c * tot[2]);
            ka.ai = (real)(c * tot[3]);
            ka.rr = (real)(c * tot[0]);
            ka.ri = (real)(c * tot[1]);
            ka.pad = 0;
            ((KAdj<real>*)kconst)[l] = ka;
        }
    }
}

template <typename real>
static hipError_t launch_rho_t(irbe_ctx* h, const void* grad, bool adj)
{
    const int64_t n = h->cfg.n_atoms;
    const int P = h->cfg.p_kspace;
    if (adj) {
        using S = RhoShape<real, true>;
        const int64_t nb = blocks_for(n, kBlock * S::atoms);
        const dim3 grid((unsigned)nb, (unsigned)((P + S::chunk - 1) / S::chunk));
        k_rho_partial<real, true><<<grid, kBlock, 0, h->stream>>>(n, P, h->sq, (const real*)h->q_orig, h->kvec,
                                                                   h->kcoef, (const real*)grad, h->rho_part);
        k_rho_final<real, true><<<P, kReduceBlock, 0, h->stream>>>(nb, h->rho_part, h->kcoef, h->rho, h->Avec,
                                                                    h->kadj);
    } else {
        using S = RhoShape<real, false>;
        const int64_t nb = blocks_for(n, kBlock * S::atoms);
        const dim3 grid((unsigned)nb, (unsigned)((P + S::chunk - 1) / S::chunk));
        k_rho_partial<real, false><<<grid, kBlock, 0, h->stream>>>(n, P, h->sq, (const real*)h->q_orig, h->kvec,
                                                                    h->kcoef, nullptr, h->rho_part);
        k_rho_final<real, false><<<P, kReduceBlock, 0, h->stream>>>(nb, h->rho_part, h->kcoef, h->rho, h->Avec,
                                                                     h->kforce);
    }
    return hipGetLastError();
}

hipError_t launch_rho(irbe_ctx* h, const void* grad, bool with_adjoint)
{
    return h->fp64 ? launch_rho_t<double>(h, grad, with_adjoint) : launch_rho_t<float>(h, grad, with_adjoint);
}

// Per atom (caller order): F_i = F_i^sr - F^corr + F_i^long,* with
// F_i^long,* = -q_i sum_l k_l (cos th a_l - sin th b_l), a_l = ke c_l Im rho_l,
// b_l = ke c_l Re rho_l, so that Im(e^{-i th} rho) = cos th Im rho - sin th Re rho.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_kspace_forces(int64_t n, int P, const uint4* __restrict__ sq,
                                                          const real* __restrict__ q, const int32_t* __restrict__ rank,
                                                          const real* __restrict__ fsr, const int4* __restrict__ kvec,
                                                          const KForce<real>* __restrict__ kf,
                                                          const double* __restrict__ fcorr, real* __restrict__ force)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 s = sq[i];
    real fx = 0, fy = 0, fz = 0;
    for (int l = 0; l < P; ++l) {
        const int4 m = kvec[l];
        const KForce<real> c = kf[l];
        real sn, cs;
        Math<real>::sincos_rev(phase_rev<real>(m.x, m.y, m.z, s.x, s.y, s.z), &sn, &cs);
        const real g = cs * c.a - sn * c.b;
        fx += g * c.kx;
        fy += g * c.ky;
        fz += g * c.kz;
    }
    const real qi = q[i];
    const int64_t k = rank[i];
    force[3 * i + 0] = fsr[3 * k + 0] - (real)fcorr[0] - qi * fx;
    force[3 * i + 1] = fsr[3 * k + 1] - (real)fcorr[1] - qi * fy;
    force[3 * i + 2] = fsr[3 * k + 2] - (real)fcorr[2] - qi * fz;
}

hipError_t launch_kspace_forces(irbe_ctx* h, void* force)
{
    const int64_t n = h->cfg.n_atoms;
    const unsigned nb = (unsigned)blocks_for(n, kBlock);
    if (h->fp64)
        k_kspace_forces<double><<<nb, kBlock, 0, h->stream>>>(n, h->cfg.p_kspace, h->sq, (const double*)h->q_orig,
                                                              h->rank, (const double*)h->fsr, h->kvec,
                                                              (const KForce<double>*)h->kforce, h->fcorr,
                                                              (double*)force);
    else
        k_kspace_forces<float><<<nb, kBlock, 0, h->stream>>>(n, h->cfg.p_kspace, h->sq, (const float*)h->q_orig,
                                                             h->rank, (const float*)h->fsr, h->kvec,
                                                             (const KForce<float>*)h->kforce, h->fcorr,
                                                             (float*)force);
    return hipGetLastError();
}

// ev[0..10] = U_coul, U_lj, U_long, U_self, U_excl, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz.
// U_long* = sum_l (c_l / 2) |rho_l|^2 (c_l carries ke (S/p) 4 pi/(V k^2)); its
// virial U_l (delta_ab - 2 k_a k_b (1/k^2 + 1/(4 alpha))).
__global__ __launch_bounds__(kReduceBlock) void k_energy_finalize(int P, const double* __restrict__ kcoef,
                                                                  const double* __restrict__ rho,
                                                                  const double* __restrict__ ev_pair,
                                                                  const double* __restrict__ sumq2, double self_coef,
                                                                  double inv_4alpha, double* __restrict__ ev)
{
    __shared__ double lds[7 * (kReduceBlock / 64)];
    double vals[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int l = threadIdx.x; l < P; l += kReduceBlock) {
        const double kx = kcoef[4 * l], ky = kcoef[4 * l + 1], kz = kcoef[4 * l + 2], c = kcoef[4 * l + 3];
        const double k2 = kx * kx + ky * ky + kz * kz;
        const double u = 0.5 * c * (rho[2 * l] * rho[2 * l] + rho[2 * l + 1] * rho[2 * l + 1]);
        const double g = 2.0 * (1.0 / k2 + inv_4alpha);
        vals[0] += u;
        vals[1] += u * (1.0 - g * kx * kx);
        vals[2] += u * (1.0 - g * ky * ky);
        vals[3] += u * (1.0 - g * kz * kz);
        vals[4] += -u * g * kx * ky;
        vals[5] += -u * g * kx * kz;
        vals[6] += -u * g * ky * kz;
    }
    double out;
    block_sum_vec<7, kReduceBlock>(vals, lds, threadIdx.x, out);
    __shared__ double tot[7];
    if (threadIdx.x < 7) tot[threadIdx.x] = out;
    __syncthreads();
    if (threadIdx.x == 0) {
        ev[0] = ev_pair[3];
        ev[1] = ev_pair[4];
        ev[2] = tot[0];
        ev[3] = self_coef * sumq2[0];
        ev[4] = ev_pair[5];
        for (int c = 0; c < 6; ++c) ev[5 + c] = ev_pair[6 + c] + tot[1 + c];
    }
}

hipError_t launch_energy_finalize(irbe_ctx* h, double* ev)
{
    const double beta = h->cfg.ewald_beta;
    const double self_coef = -h->cfg.coulomb_k * beta / 1.7724538509055160273;
    k_energy_finalize<<<1, kReduceBlock, 0, h->stream>>>(h->cfg.p_kspace, h->kcoef, h->rho, h->ev_pair, h->sumq2,
                                                         self_coef, 1.0 / (4.0 * beta * beta), ev);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Backward.
// ---------------------------------------------------------------------------

// dL/dF into cell order, and per-block FP64 sums for mean(G).
template <typename real>
__global__ __launch_bounds__(kBlock) void k_gather_grad(int64_t n, const int32_t* __restrict__ perm,
                                                        const real* __restrict__ G, real* __restrict__ gs,
                                                        double* __restrict__ part)
{
    __shared__ double lds[3 * (kBlock / 64)];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double vals[3] = {0, 0, 0};
    if (k < n) {
        const int64_t i = perm[k];
        const real gx = G[3 * i], gy = G[3 * i + 1], gz = G[3 * i + 2];
        gs[3 * k] = gx;
        gs[3 * k + 1] = gy;
        gs[3 * k + 2] = gz;
        vals[0] = (double)gx;
        vals[1] = (double)gy;
        vals[2] = (double)gz;
    }
    double out;
    block_sum_vec<3, kBlock>(vals, lds, threadIdx.x, out);
    if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = out;
}

__global__ __launch_bounds__(kReduceBlock) void k_mean3(int64_t nb, const double* __restrict__ part, int64_t n,
                                                        double* __restrict__ mean)
{
    __shared__ double lds[3 * (kReduceBlock / 64)];
    double vals[3] = {0, 0, 0};
    for (int64_t b = threadIdx.x; b < nb; b += kReduceBlock)
        for (int c = 0; c < 3; ++c) vals[c] += part[b * 3 + c];
    double out;
    block_sum_vec<3, kReduceBlock>(vals, lds, threadIdx.x, out);
    if (threadIdx.x < 3) mean[threadIdx.x] = out / (double)n;
}

hipError_t launch_gather_grad(irbe_ctx* h, const void* grad)
{
    const int64_t n = h->cfg.n_atoms;
    const int64_t nb = blocks_for(n, kBlock);
    if (h->fp64)
        k_gather_grad<double><<<(unsigned)nb, kBlock, 0, h->stream>>>(n, h->perm, (const double*)grad, (double*)h->gs,
                                                                      h->gpart);
    else
        k_gather_grad<float><<<(unsigned)nb, kBlock, 0, h->stream>>>(n, h->perm, (const float*)grad, (float*)h->gs,
                                                                     h->gpart);
    k_mean3<<<1, kReduceBlock, 0, h->stream>>>(nb, h->gpart, n, h->gmean);
    return hipGetLastError();
}

// Per atom (caller order): the k-space adjoint plus the short-range parts.
//   dL/dr_n = -ke q_n sum_l c_l k_l [Re(e^{i th} conj A_l) - g_nl Re(e^{-i th} rho_l)]
//   dL/dq_n = -ke sum_l c_l [Im(e^{i th} conj A_l) + g_nl Im(e^{-i th} rho_l)]
template <typename real>
__global__ __launch_bounds__(kBlock) void k_kspace_adjoint(int64_t n, int P, const uint4* __restrict__ sq,
                                                           const real* __restrict__ q, const real* __restrict__ G,
                                                           const int32_t* __restrict__ rank,
                                                           const int4* __restrict__ kvec,
                                                           const KAdj<real>* __restrict__ ka,
                                                           const real* __restrict__ gself,
                                                           const real* __restrict__ gscat,
                                                           const real* __restrict__ gqself,
                                                           const real* __restrict__ gqscat, real* __restrict__ gpos,
                                                           real* __restrict__ gq)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 s = sq[i];
    const real gx = G[3 * i], gy = G[3 * i + 1], gz = G[3 * i + 2];
    real px = 0, py = 0, pz = 0, pq = 0;
    for (int l = 0; l < P; ++l) {
        const int4 m = kvec[l];
        const KAdj<real> c = ka[l];
        real sn, cs;
        Math<real>::sincos_rev(phase_rev<real>(m.x, m.y, m.z, s.x, s.y, s.z), &sn, &cs);
        const real g = gx * c.kx + gy * c.ky + gz * c.kz;
        const real eA_re = cs * c.ar + sn * c.ai;
        const real eA_im = sn * c.ar - cs * c.ai;
        const real er_re = cs * c.rr + sn * c.ri;
        const real er_im = cs * c.ri - sn * c.rr;
        const real t = eA_re - g * er_re;
        px += t * c.kx;
        py += t * c.ky;
        pz += t * c.kz;
        pq += eA_im + g * er_im;
    }
    const real qi = q[i];
    const int64_t k = rank[i];
    gpos[3 * i + 0] = gself[3 * k + 0] + gscat[3 * k + 0] - qi * px;
    gpos[3 * i + 1] = gself[3 * k + 1] + gscat[3 * k + 1] - qi * py;
    gpos[3 * i + 2] = gself[3 * k + 2] + gscat[3 * k + 2] - qi * pz;
    if (gq) gq[i] = gqself[k] + gqscat[k] - pq;
}

// LJ table gradients: fixed-order two-stage sum of the per-block partials
// (slices of contiguous blocks, then the slices).
constexpr int kLjSlices = 256;

__global__ __launch_bounds__(kReduceBlock) void k_lj_reduce1(int64_t nb, const double* __restrict__ part,
                                                             double* __restrict__ slices)
{
    constexpr int NLJ = 2 * kMaxTypesGrad * kMaxTypesGrad;
    __shared__ double lds[NLJ * (kReduceBlock / 64)];
    const int64_t per = (nb + kLjSlices - 1) / kLjSlices;
    const int64_t b0 = blockIdx.x * per, b1 = min(nb, b0 + per);
    double vals[NLJ];
    for (int v = 0; v < NLJ; ++v) vals[v] = 0.0;
    for (int64_t b = b0 + threadIdx.x; b < b1; b += kReduceBlock)
        for (int v = 0; v < NLJ; ++v) vals[v] += part[b * NLJ + v];
    double o;
    block_sum_vec<NLJ, kReduceBlock>(vals, lds, threadIdx.x, o);
    if (threadIdx.x < NLJ) slices[blockIdx.x * NLJ + threadIdx.x] = o;
}

__global__ __launch_bounds__(kReduceBlock) void k_lj_reduce2(const double* __restrict__ slices, int n_types,
                                                             double* __restrict__ out)
{
    constexpr int NLJ = 2 * kMaxTypesGrad * kMaxTypesGrad;
    __shared__ double lds[NLJ * (kReduceBlock / 64)];
    double vals[NLJ];
    for (int v = 0; v < NLJ; ++v) vals[v] = 0.0;
    for (int b = threadIdx.x; b < kLjSlices; b += kReduceBlock)
        for (int v = 0; v < NLJ; ++v) vals[v] += slices[b * NLJ + v];
    double o;
    block_sum_vec<NLJ, kReduceBlock>(vals, lds, threadIdx.x, o);
    if (threadIdx.x < NLJ) {
        const int half = kMaxTypesGrad * kMaxTypesGrad;
        const int which = threadIdx.x / half;  // 0 sigma, 1 eps
        const int e = threadIdx.x % half;
        const int a = e / kMaxTypesGrad, t = e % kMaxTypesGrad;
        if (a < n_types && t < n_types) out[which * n_types * n_types + a * n_types + t] = o;
    }
}

hipError_t launch_kspace_adjoint(irbe_ctx* h, const void* grad, void* grad_pos, void* grad_q, double* grad_lj)
{
    const int64_t n = h->cfg.n_atoms;
    const unsigned nb = (unsigned)blocks_for(n, kBlock);
    if (h->fp64)
        k_kspace_adjoint<double><<<nb, kBlock, 0, h->stream>>>(
            n, h->cfg.p_kspace, h->sq, (const double*)h->q_orig, (const double*)grad, h->rank, h->kvec,
            (const KAdj<double>*)h->kadj, (const double*)h->gself, (const double*)h->gscat, (const double*)h->gqself,
            (const double*)h->gqscat, (double*)grad_pos, (double*)grad_q);
    else
        k_kspace_adjoint<float><<<nb, kBlock, 0, h->stream>>>(
            n, h->cfg.p_kspace, h->sq, (const float*)h->q_orig, (const float*)grad, h->rank, h->kvec,
            (const KAdj<float>*)h->kadj, (const float*)h->gself, (const float*)h->gscat, (const float*)h->gqself,
            (const float*)h->gqscat, (float*)grad_pos, (float*)grad_q);
    if (grad_lj) {
        k_lj_reduce1<<<kLjSlices, kReduceBlock, 0, h->stream>>>(h->adj_nb, h->ljpart, h->lj_slices);
        k_lj_reduce2<<<1, kReduceBlock, 0, h->stream>>>(h->lj_slices, h->cfg.n_types, grad_lj);
    }
    return hipGetLastError();
}

}  // namespace irbe
