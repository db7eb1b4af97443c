// Short-range part of the force (Sec. 2.3) and its adjoint.
//
// Forward, per atom i (cell order), Eqs. (2.10)-(2.12):
//   F_i = sum_{j in C(i)} f_ij + w_i sum_{j in B(i)} f_ij + F_i^excl
// with B(i) a batch of p_shell ranks of S(i) drawn without replacement by
// Floyd's algorithm from the Philox word stream of (seed, step, caller id of
// i), w_i = N_S / p_shell (all members and w_i = 1 when N_S <= p_shell). The
// per-block FP64 sums of the uncorrected short-range force give F^corr.
// Full-list mode: one list of every pair within r_shell, weight 1.
#include "irbe_device.hpp"
#include "irbe_internal.hpp"

namespace irbe {

template <typename real>
struct PairParams {
    real quantum;   // L / 2^32
    real beta;
    real cgauss;    // 2 beta / sqrt(pi)
    real ke;
};

template <typename real>
__device__ __forceinline__ void separation(uint4 a, uint4 b, real quantum, real& dx, real& dy, real& dz)
{
    dx = (real)(int32_t)(b.x - a.x) * quantum;
    dy = (real)(int32_t)(b.y - a.y) * quantum;
    dz = (real)(int32_t)(b.z - a.z) * quantum;
}

// phi of f_ij = phi r_ij (Eq. (2.10)) and, when EV, the pair energies.
template <typename real, bool EV>
__device__ __forceinline__ real pair_phi(real r2, real qq, const LJ<real>& lj, const PairParams<real>& pp, real& uc,
                                         real& ul)
{
    using M = Math<real>;
    const real rinv = M::rsqrt_(r2);
    const real r = r2 * rinv;
    const real br = pp.beta * r;
    const real ex = M::exp_(-br * br);
    const real ec = M::erfc_(br);
    const real rinv2 = rinv * rinv;
    const real r6 = rinv2 * rinv2 * rinv2;
    real phi = -qq * rinv2 * (ec * rinv + pp.cgauss * ex);
    phi -= r6 * rinv2 * (lj.a12 * r6 - lj.b6);
    if (EV) {
        uc = qq * ec * rinv;
        ul = r6 * (lj.c12 * r6 - lj.c6);
    }
    return phi;
}

// psi of the excluded-pair correction f = psi r_ij and its energy.
template <typename real, bool EV>
__device__ __forceinline__ real excl_psi(real r2, real qq, const PairParams<real>& pp, real& ux)
{
    using M = Math<real>;
    const real rinv = M::rsqrt_(r2);
    const real r = r2 * rinv;
    const real br = pp.beta * r;
    const real ex = M::exp_(-br * br);
    const real ef = M::erf_(br);
    const real rinv2 = rinv * rinv;
    if (EV) ux = -qq * ef * rinv;
    return -qq * rinv2 * (pp.cgauss * ex - ef * rinv);
}

template <typename real>
struct Acc3 {
    real x = 0, y = 0, z = 0;
};

template <typename real, bool FULL, bool EV, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_pair_forces(
    int64_t n, PairParams<real> pp, const uint4* __restrict__ spos, const real* __restrict__ sqr,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ rank, const int32_t* __restrict__ core,
    const int32_t* __restrict__ ncore, int cap_core, const int32_t* __restrict__ shell,
    const int32_t* __restrict__ nshell, int cap_shell, const int32_t* __restrict__ xoff,
    const int32_t* __restrict__ xidx, const LJ<real>* __restrict__ lj_g, int n_types, int p_shell, uint64_t seed,
    uint64_t step, int bm_words, real* __restrict__ fsr, double* __restrict__ part)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    LJ<real>* lj = (LJ<real>*)smem_raw;
    const int nt2 = n_types * n_types;
    uint32_t* bitmap = (uint32_t*)(smem_raw + ((sizeof(LJ<real>) * nt2 + 15) / 16) * 16);
    __shared__ double red[kPairPartials * (BLOCK / 64)];
    for (int t = threadIdx.x; t < nt2; t += BLOCK) lj[t] = lj_g[t];
    __syncthreads();

    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    Acc3<real> fc, fs, fx;
    real uc_c = 0, ul_c = 0, uc_s = 0, ul_s = 0, ux = 0;
    real vc[6] = {0, 0, 0, 0, 0, 0}, vs[6] = {0, 0, 0, 0, 0, 0}, vx[6] = {0, 0, 0, 0, 0, 0};
    real w = 1;
    if (k < n) {
        const uint4 si = spos[k];
        const real qi = sqr[k] * pp.ke;
        const LJ<real>* lrow = lj + (int)si.w * n_types;
        // core pairs
        const int nc = ncore[k];
        const int32_t* crow = core + k * (int64_t)cap_core;
        for (int c = 0; c < nc; ++c) {
            const int j = crow[c];
            const uint4 sj = spos[j];
            real dx, dy, dz;
            separation(si, sj, pp.quantum, dx, dy, dz);
            const real r2 = dx * dx + dy * dy + dz * dz;
            real uc, ul;
            const real phi = pair_phi<real, EV>(r2, qi * sqr[j], lrow[sj.w], pp, uc, ul);
            fc.x += phi * dx;
            fc.y += phi * dy;
            fc.z += phi * dz;
            if (EV) {
                uc_c += uc;
                ul_c += ul;
                vc[0] += phi * dx * dx; vc[1] += phi * dy * dy; vc[2] += phi * dz * dz;
                vc[3] += phi * dx * dy; vc[4] += phi * dx * dz; vc[5] += phi * dy * dz;
            }
        }
        // shell: every member, or the Floyd batch
        const int ns = nshell[k];
        const int32_t* srow = shell + k * (int64_t)cap_shell;
        const bool sample = !FULL && ns > p_shell;
        const int cnt = sample ? p_shell : ns;
        WordStream st(seed, step, (uint32_t)perm[k], kTagShell);
        if (sample) {
            w = (real)((double)ns / (double)p_shell);
            const int words = (ns + 31) >> 5;
            for (int t = 0; t < words; ++t) bitmap[t * BLOCK + threadIdx.x] = 0u;
        }
        for (int c = 0; c < cnt; ++c) {
            int v = c;
            if (sample) {
                const int t = ns - p_shell + c;
                const int r = (int)st.below((uint32_t)t + 1u);
                uint32_t* wr = &bitmap[(r >> 5) * BLOCK + threadIdx.x];
                const bool taken = (*wr >> (r & 31)) & 1u;
                v = taken ? t : r;
                bitmap[(v >> 5) * BLOCK + threadIdx.x] |= 1u << (v & 31);
            }
            const int j = srow[v];
            const uint4 sj = spos[j];
            real dx, dy, dz;
            separation(si, sj, pp.quantum, dx, dy, dz);
            const real r2 = dx * dx + dy * dy + dz * dz;
            real uc, ul;
            const real phi = pair_phi<real, EV>(r2, qi * sqr[j], lrow[sj.w], pp, uc, ul);
            fs.x += phi * dx;
            fs.y += phi * dy;
            fs.z += phi * dz;
            if (EV) {
                uc_s += uc;
                ul_s += ul;
                vs[0] += phi * dx * dx; vs[1] += phi * dy * dy; vs[2] += phi * dz * dz;
                vs[3] += phi * dx * dy; vs[4] += phi * dx * dz; vs[5] += phi * dy * dz;
            }
        }
        // excluded pairs: remove their reciprocal-space erf(beta r)/r interaction
        const int ic = perm[k];
        for (int x = xoff[ic]; x < xoff[ic + 1]; ++x) {
            const int j = rank[xidx[x]];
            const uint4 sj = spos[j];
            real dx, dy, dz;
            separation(si, sj, pp.quantum, dx, dy, dz);
            const real r2 = dx * dx + dy * dy + dz * dz;
            real u;
            const real psi = excl_psi<real, EV>(r2, qi * sqr[j], pp, u);
            fx.x += psi * dx;
            fx.y += psi * dy;
            fx.z += psi * dz;
            if (EV) {
                ux += u;
                vx[0] += psi * dx * dx; vx[1] += psi * dy * dy; vx[2] += psi * dz * dz;
                vx[3] += psi * dx * dy; vx[4] += psi * dx * dz; vx[5] += psi * dy * dz;
            }
        }
        const real px = fc.x + w * fs.x, py = fc.y + w * fs.y, pz = fc.z + w * fs.z;
        fsr[3 * k + 0] = px + fx.x;
        fsr[3 * k + 1] = py + fx.y;
        fsr[3 * k + 2] = pz + fx.z;
        fc.x = px; fc.y = py; fc.z = pz;
    }
    double vals[kPairPartials];
    vals[0] = (double)fc.x;
    vals[1] = (double)fc.y;
    vals[2] = (double)fc.z;
    if (EV) {
        vals[3] = 0.5 * ((double)uc_c + (double)w * (double)uc_s);
        vals[4] = 0.5 * ((double)ul_c + (double)w * (double)ul_s);
        vals[5] = 0.5 * (double)ux;
        for (int c = 0; c < 6; ++c) vals[6 + c] = -0.5 * ((double)vc[c] + (double)w * (double)vs[c] + (double)vx[c]);
    } else {
        for (int c = 3; c < 12; ++c) vals[c] = 0.0;
    }
    for (int c = 12; c < kPairPartials; ++c) vals[c] = 0.0;
    double out;
    block_sum_vec<12, BLOCK>(vals, red, threadIdx.x, out);
    if (threadIdx.x < 12) part[blockIdx.x * (int64_t)kPairPartials + threadIdx.x] = out;
}

// Reduce the per-block partials in a fixed order: ev_pair[0..11] = totals,
// fcorr = (sum of the uncorrected short-range force) / N when rbl.
__global__ __launch_bounds__(kReduceBlock) void k_pair_reduce(int64_t nb, const double* __restrict__ part, int64_t n,
                                                              int rbl, double* __restrict__ ev_pair,
                                                              double* __restrict__ fcorr)
{
    __shared__ double lds[12 * (kReduceBlock / 64)];
    double vals[12];
    for (int c = 0; c < 12; ++c) vals[c] = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += kReduceBlock)
        for (int c = 0; c < 12; ++c) vals[c] += part[b * kPairPartials + c];
    double out;
    block_sum_vec<12, kReduceBlock>(vals, lds, threadIdx.x, out);
    if (threadIdx.x < 12) ev_pair[threadIdx.x] = out;
    if (threadIdx.x < 3) fcorr[threadIdx.x] = rbl ? out / (double)n : 0.0;
}

template <typename real, bool FULL, bool EV, int BLOCK>
static void launch_pair_t(irbe_ctx* h, uint64_t step, int bm_words, size_t lds)
{
    const int64_t n = h->cfg.n_atoms;
    PairParams<real> pp;
    pp.quantum = (real)h->geo.quantum;
    pp.beta = (real)h->cfg.ewald_beta;
    pp.cgauss = (real)(2.0 * h->cfg.ewald_beta / 1.7724538509055160273);
    pp.ke = (real)h->cfg.coulomb_k;
    const unsigned nb = (unsigned)blocks_for(n, BLOCK);
    k_pair_forces<real, FULL, EV, BLOCK><<<nb, BLOCK, lds, h->stream>>>(
        n, pp, h->spos, (const real*)h->sq_r, h->perm, h->rank, h->core, h->ncore, h->cap_core, h->shell, h->nshell,
        h->cap_shell, h->xoff, h->xidx, (const LJ<real>*)h->lj, h->cfg.n_types, h->cfg.p_shell, h->cfg.seed, step,
        bm_words, (real*)h->fsr, h->pair_part);
    h->pair_nb = nb;
}

hipError_t launch_pair_reduce(irbe_ctx* h)
{
    k_pair_reduce<<<1, kReduceBlock, 0, h->stream>>>(h->pair_nb, h->pair_part, h->cfg.n_atoms, h->full_list ? 0 : 1,
                                                     h->ev_pair, h->fcorr);
    return hipGetLastError();
}

template <typename real>
static hipError_t launch_pair_r(irbe_ctx* h, uint64_t step, bool ev)
{
    const int words = h->full_list ? 0 : (h->max_shell + 31) / 32;
    const size_t lj_bytes = ((sizeof(LJ<real>) * h->cfg.n_types * h->cfg.n_types + 15) / 16) * 16;
    const size_t lds256 = lj_bytes + (size_t)words * 256 * 4;
    const size_t lds64 = lj_bytes + (size_t)words * 64 * 4;
    const bool big = lds256 > 48 * 1024;
    if (big && lds64 > 64 * 1024) return hipErrorInvalidValue;
    if (h->full_list) {
        if (ev) launch_pair_t<real, true, true, 256>(h, step, words, lds256);
        else launch_pair_t<real, true, false, 256>(h, step, words, lds256);
    } else if (!big) {
        if (ev) launch_pair_t<real, false, true, 256>(h, step, words, lds256);
        else launch_pair_t<real, false, false, 256>(h, step, words, lds256);
    } else {
        if (ev) launch_pair_t<real, false, true, 64>(h, step, words, lds64);
        else launch_pair_t<real, false, false, 64>(h, step, words, lds64);
    }
    return hipGetLastError();
}

hipError_t launch_pair_forces(irbe_ctx* h, uint64_t step, bool ev)
{
    return h->fp64 ? launch_pair_r<double>(h, step, ev) : launch_pair_r<float>(h, step, ev);
}

// Batch ranks of every atom (debug read-back): ranks_dev[k * stride + t] for
// the atom in cell-order slot k, in draw order.
__global__ __launch_bounds__(kBlock) void k_batch_debug(int64_t n, const int32_t* __restrict__ perm,
                                                        const int32_t* __restrict__ nshell, int p_shell, uint64_t seed,
                                                        uint64_t step, int32_t* __restrict__ ranks, int stride,
                                                        uint32_t* __restrict__ bits, int words)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int ns = nshell[k];
    int32_t* out = ranks + k * (int64_t)stride;
    if (p_shell <= 0 || ns <= p_shell) {
        for (int t = 0; t < ns; ++t) out[t] = t;
        return;
    }
    uint32_t* bm = bits + k * (int64_t)words;
    for (int t = 0; t < words; ++t) bm[t] = 0u;
    WordStream st(seed, step, (uint32_t)perm[k], kTagShell);
    for (int c = 0; c < p_shell; ++c) {
        const int t = ns - p_shell + c;
        const int r = (int)st.below((uint32_t)t + 1u);
        const bool taken = (bm[r >> 5] >> (r & 31)) & 1u;
        const int v = taken ? t : r;
        bm[v >> 5] |= 1u << (v & 31);
        out[c] = v;
    }
}

hipError_t launch_batch_debug(irbe_ctx* h, uint64_t step, int32_t* ranks_dev, int32_t stride)
{
    const int64_t n = h->cfg.n_atoms;
    const int words = (h->max_shell + 31) / 32 + 1;
    uint32_t* bits = nullptr;
    hipError_t e = hipMalloc(&bits, (size_t)n * words * 4);
    if (e != hipSuccess) return e;
    k_batch_debug<<<(unsigned)blocks_for(n, kBlock), kBlock, 0, h->stream>>>(
        n, h->perm, h->nshell, h->cfg.p_shell, h->cfg.seed, step, ranks_dev, stride, bits, words);
    e = hipStreamSynchronize(h->stream);
    hipFree(bits);
    return e;
}

// ---------------------------------------------------------------------------
// Adjoint of the short-range force (vector-Jacobian product with G = dL/dF at
// fixed lists and batches). With f_ij = phi(r) r_ij, J = phi I + (phi'/r) r r^T
// is symmetric and even in r_ij, so for the symmetric sets (C(i), the full list,
// the excluded pairs) the gradient is gathered per atom:
//   dL/dr_i += sum_j J (G'_j - G'_i),  dL/dq_i += sum_j (ke q_j a(r)) r_ij.(G'_j - G'_i)
// where a(r) is the Coulomb factor of phi / (-ke q_i q_j). The sampled shell
// terms are one-sided: dL/dr_i -= w J G'_i and dL/dr_j += w J G'_i (scattered
// with atomics), and likewise for the charges. G' = G - mean(G) for the pair
// terms when the momentum correction is applied; excluded pairs use G.
// LJ table gradients are accumulated per (t_i, t_j) entry in FP64.
// ---------------------------------------------------------------------------
template <typename real>
struct PairGrad {
    real phi, dphi_r;   // phi and phi'(r)/r
    real a_coul;        // erfc/r^3 + 2b e^{-b^2 r^2}/(sqrt(pi) r^2): phi_coul = -qq a_coul
    real c_lj;          // 48 s^12/r^14 - 24 s^6/r^8: phi_lj = -eps c_lj
    real dc_dsig;       // d c_lj / d sigma
};

template <typename real>
__device__ __forceinline__ PairGrad<real> pair_grad(real r2, real qq, real sig, real eps, const PairParams<real>& pp)
{
    using M = Math<real>;
    const real rinv = M::rsqrt_(r2);
    const real r = r2 * rinv;
    const real br = pp.beta * r;
    const real ex = M::exp_(-br * br);
    const real ec = M::erfc_(br);
    const real rinv2 = rinv * rinv;
    const real rinv3 = rinv2 * rinv;
    const real A = ec * rinv3;
    const real B = pp.cgauss * ex * rinv2;
    const real dA = -pp.cgauss * ex * rinv3 - (real)3 * ec * rinv3 * rinv;
    const real dB = -pp.cgauss * ex * ((real)2 * pp.beta * pp.beta * rinv + (real)2 * rinv3);
    const real s2 = sig * sig;
    const real s6 = s2 * s2 * s2;
    const real s12 = s6 * s6;
    const real r6 = rinv2 * rinv2 * rinv2;
    const real C = rinv2 * r6 * ((real)48 * s12 * r6 - (real)24 * s6);
    const real dC = rinv * rinv2 * r6 * ((real)-672 * s12 * r6 + (real)192 * s6);
    const real dCs = sig != (real)0 ? rinv2 * r6 * ((real)576 * s12 * r6 - (real)144 * s6) / sig : (real)0;
    PairGrad<real> g;
    g.a_coul = A + B;
    g.phi = -qq * (A + B) - eps * C;
    g.dphi_r = (-qq * (dA + dB) - eps * dC) * rinv;
    g.c_lj = C;
    g.dc_dsig = dCs;
    return g;
}

template <typename real>
__device__ __forceinline__ void excl_grad(real r2, real qq, const PairParams<real>& pp, real& psi, real& dpsi_r,
                                          real& a_x)
{
    using M = Math<real>;
    const real rinv = M::rsqrt_(r2);
    const real r = r2 * rinv;
    const real br = pp.beta * r;
    const real ex = M::exp_(-br * br);
    const real ef = M::erf_(br);
    const real rinv2 = rinv * rinv;
    const real rinv3 = rinv2 * rinv;
    const real Bx = pp.cgauss * ex * rinv2;
    const real E = ef * rinv3;
    const real dBx = -pp.cgauss * ex * ((real)2 * pp.beta * pp.beta * rinv + (real)2 * rinv3);
    const real dE = pp.cgauss * ex * rinv3 - (real)3 * ef * rinv3 * rinv;
    a_x = Bx - E;
    psi = -qq * a_x;
    dpsi_r = -qq * (dBx - dE) * rinv;
}

template <typename real>
__device__ __forceinline__ void load3(const real* p, int64_t k, real& x, real& y, real& z)
{
    x = p[3 * k];
    y = p[3 * k + 1];
    z = p[3 * k + 2];
}

template <typename real, bool FULL, bool WANT_LJ, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_pair_adjoint(
    int64_t n, PairParams<real> pp, const uint4* __restrict__ spos, const real* __restrict__ sqr,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ rank, const int32_t* __restrict__ core,
    const int32_t* __restrict__ ncore, int cap_core, const int32_t* __restrict__ shell,
    const int32_t* __restrict__ nshell, int cap_shell, const int32_t* __restrict__ xoff,
    const int32_t* __restrict__ xidx, const real* __restrict__ ljraw_g, int n_types, int p_shell, uint64_t seed,
    uint64_t step, const real* __restrict__ gs, const double* __restrict__ gmean_d, real* __restrict__ gself,
    real* __restrict__ gscat, real* __restrict__ gqself, real* __restrict__ gqscat, double* __restrict__ ljpart)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    real* ljraw = (real*)smem_raw;  // sigma[nt2], eps[nt2]
    const int nt2 = n_types * n_types;
    uint32_t* bitmap = (uint32_t*)(smem_raw + ((sizeof(real) * 2 * nt2 + 15) / 16) * 16);
    constexpr int NLJ = 2 * kMaxTypesGrad * kMaxTypesGrad;
    __shared__ double red[NLJ * (BLOCK / 64)];
    for (int t = threadIdx.x; t < 2 * nt2; t += BLOCK) ljraw[t] = ljraw_g[t];
    __syncthreads();

    const real mx = FULL ? (real)0 : (real)gmean_d[0];
    const real my = FULL ? (real)0 : (real)gmean_d[1];
    const real mz = FULL ? (real)0 : (real)gmean_d[2];
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double acc_sig[kMaxTypesGrad], acc_eps[kMaxTypesGrad];
#pragma unroll
    for (int t = 0; t < kMaxTypesGrad; ++t) acc_sig[t] = acc_eps[t] = 0.0;
    int ti = 0;
    if (k < n) {
        const uint4 si = spos[k];
        ti = (int)si.w;
        const real qi = sqr[k];
        const real ke = pp.ke;
        real gx, gy, gz;
        load3(gs, k, gx, gy, gz);
        const real pgx = gx - mx, pgy = gy - my, pgz = gz - mz;  // G'_i
        real rx = 0, ry = 0, rz = 0, rq = 0;
        // symmetric part: core pairs (RBL) or the whole list (full-list mode)
        for (int list = 0; list < 2; ++list) {
            const bool sym = list == 0 || FULL;
            const int nc = list == 0 ? ncore[k] : nshell[k];
            if (!sym) break;
            const int32_t* row = list == 0 ? core + k * (int64_t)cap_core : shell + k * (int64_t)cap_shell;
            for (int c = 0; c < nc; ++c) {
                const int j = row[c];
                const uint4 sj = spos[j];
                real dx, dy, dz;
                separation(si, sj, pp.quantum, dx, dy, dz);
                const real r2 = dx * dx + dy * dy + dz * dz;
                const int tp = ti * n_types + (int)sj.w;
                const real sig = ljraw[tp], eps = ljraw[nt2 + tp];
                const real qj = sqr[j];
                const PairGrad<real> g = pair_grad(r2, ke * qi * qj, sig, eps, pp);
                real hx, hy, hz;
                load3(gs, (int64_t)j, hx, hy, hz);
                const real ex_ = hx - mx - pgx, ey_ = hy - my - pgy, ez_ = hz - mz - pgz;  // G'_j - G'_i
                const real gd = dx * ex_ + dy * ey_ + dz * ez_;
                rx += g.phi * ex_ + g.dphi_r * dx * gd;
                ry += g.phi * ey_ + g.dphi_r * dy * gd;
                rz += g.phi * ez_ + g.dphi_r * dz * gd;
                rq += ke * qj * g.a_coul * gd;
                if (WANT_LJ) {
                    const real gdi = dx * pgx + dy * pgy + dz * pgz;
                    const int tj = (int)sj.w;
#pragma unroll
                    for (int t = 0; t < kMaxTypesGrad; ++t)
                        if (t == tj) {
                            acc_sig[t] += (double)(-eps * g.dc_dsig * gdi);
                            acc_eps[t] += (double)(-g.c_lj * gdi);
                        }
                }
            }
        }
        if (!FULL) {
            // sampled shell pairs, one-sided
            const int ns = nshell[k];
            const int32_t* srow = shell + k * (int64_t)cap_shell;
            const bool sample = ns > p_shell;
            const int cnt = sample ? p_shell : ns;
            const real w = sample ? (real)((double)ns / (double)p_shell) : (real)1;
            WordStream st(seed, step, (uint32_t)perm[k], kTagShell);
            if (sample) {
                const int words = (ns + 31) >> 5;
                for (int t = 0; t < words; ++t) bitmap[t * BLOCK + threadIdx.x] = 0u;
            }
            for (int c = 0; c < cnt; ++c) {
                int v = c;
                if (sample) {
                    const int t = ns - p_shell + c;
                    const int r = (int)st.below((uint32_t)t + 1u);
                    const bool taken = (bitmap[(r >> 5) * BLOCK + threadIdx.x] >> (r & 31)) & 1u;
                    v = taken ? t : r;
                    bitmap[(v >> 5) * BLOCK + threadIdx.x] |= 1u << (v & 31);
                }
                const int j = srow[v];
                const uint4 sj = spos[j];
                real dx, dy, dz;
                separation(si, sj, pp.quantum, dx, dy, dz);
                const real r2 = dx * dx + dy * dy + dz * dz;
                const int tp = ti * n_types + (int)sj.w;
                const real sig = ljraw[tp], eps = ljraw[nt2 + tp];
                const real qj = sqr[j];
                const PairGrad<real> g = pair_grad(r2, ke * qi * qj, sig, eps, pp);
                const real gdi = dx * pgx + dy * pgy + dz * pgz;
                const real jx = w * (g.phi * pgx + g.dphi_r * dx * gdi);
                const real jy = w * (g.phi * pgy + g.dphi_r * dy * gdi);
                const real jz = w * (g.phi * pgz + g.dphi_r * dz * gdi);
                rx -= jx;
                ry -= jy;
                rz -= jz;
                atomicAdd(&gscat[3 * (int64_t)j + 0], jx);
                atomicAdd(&gscat[3 * (int64_t)j + 1], jy);
                atomicAdd(&gscat[3 * (int64_t)j + 2], jz);
                rq += w * (-ke * qj * g.a_coul) * gdi;
                atomicAdd(&gqscat[j], w * (-ke * qi * g.a_coul) * gdi);
                if (WANT_LJ) {
                    const int tj = (int)sj.w;
#pragma unroll
                    for (int t = 0; t < kMaxTypesGrad; ++t)
                        if (t == tj) {
                            acc_sig[t] += (double)(w * (-eps * g.dc_dsig * gdi));
                            acc_eps[t] += (double)(w * (-g.c_lj * gdi));
                        }
                }
            }
        }
        // excluded pairs (symmetric; G itself)
        const int ic = perm[k];
        for (int x = xoff[ic]; x < xoff[ic + 1]; ++x) {
            const int j = rank[xidx[x]];
            const uint4 sj = spos[j];
            real dx, dy, dz;
            separation(si, sj, pp.quantum, dx, dy, dz);
            const real r2 = dx * dx + dy * dy + dz * dz;
            const real qj = sqr[j];
            real psi, dpsi_r, a_x;
            excl_grad(r2, ke * qi * qj, pp, psi, dpsi_r, a_x);
            real hx, hy, hz;
            load3(gs, (int64_t)j, hx, hy, hz);
            const real ex_ = hx - gx, ey_ = hy - gy, ez_ = hz - gz;
            const real gd = dx * ex_ + dy * ey_ + dz * ez_;
            rx += psi * ex_ + dpsi_r * dx * gd;
            ry += psi * ey_ + dpsi_r * dy * gd;
            rz += psi * ez_ + dpsi_r * dz * gd;
            rq += ke * qj * a_x * gd;
        }
        gself[3 * k + 0] = rx;
        gself[3 * k + 1] = ry;
        gself[3 * k + 2] = rz;
        gqself[k] = rq;
    }
    if (WANT_LJ) {
        // per-block sums of the table entries [t_i][t], sigma then eps
        double vals[NLJ];
#pragma unroll
        for (int a = 0; a < kMaxTypesGrad; ++a)
#pragma unroll
            for (int t = 0; t < kMaxTypesGrad; ++t) {
                const bool mine = (k < n) && (ti == a);
                vals[a * kMaxTypesGrad + t] = mine ? acc_sig[t] : 0.0;
                vals[kMaxTypesGrad * kMaxTypesGrad + a * kMaxTypesGrad + t] = mine ? acc_eps[t] : 0.0;
            }
        double out;
        block_sum_vec<NLJ, BLOCK>(vals, red, threadIdx.x, out);
        if (threadIdx.x < NLJ) ljpart[blockIdx.x * (int64_t)NLJ + threadIdx.x] = out;
    }
}

template <typename real, bool FULL, bool WANT_LJ, int BLOCK>
static void launch_adj_t(irbe_ctx* h, uint64_t step, size_t lds)
{
    const int64_t n = h->cfg.n_atoms;
    PairParams<real> pp;
    pp.quantum = (real)h->geo.quantum;
    pp.beta = (real)h->cfg.ewald_beta;
    pp.cgauss = (real)(2.0 * h->cfg.ewald_beta / 1.7724538509055160273);
    pp.ke = (real)h->cfg.coulomb_k;
    const unsigned nb = (unsigned)blocks_for(n, BLOCK);
    h->adj_nb = nb;
    k_pair_adjoint<real, FULL, WANT_LJ, BLOCK><<<nb, BLOCK, lds, h->stream>>>(
        n, pp, h->spos, (const real*)h->sq_r, h->perm, h->rank, h->core, h->ncore, h->cap_core, h->shell, h->nshell,
        h->cap_shell, h->xoff, h->xidx, (const real*)h->lj_raw, h->cfg.n_types, h->cfg.p_shell, h->cfg.seed, step,
        (const real*)h->gs, h->gmean, (real*)h->gself, (real*)h->gscat, (real*)h->gqself, (real*)h->gqscat,
        h->ljpart);
}

template <typename real>
static hipError_t launch_adj_r(irbe_ctx* h, uint64_t step, bool want_lj)
{
    const int words = h->full_list ? 0 : (h->max_shell + 31) / 32;
    const size_t raw_bytes = ((sizeof(real) * 2 * h->cfg.n_types * h->cfg.n_types + 15) / 16) * 16;
    const size_t lds256 = raw_bytes + (size_t)words * 256 * 4;
    const size_t lds64 = raw_bytes + (size_t)words * 64 * 4;
    const bool big = lds256 > 48 * 1024;
    if (big && lds64 > 64 * 1024) return hipErrorInvalidValue;
    if (h->full_list) {
        if (want_lj) launch_adj_t<real, true, true, 256>(h, step, lds256);
        else launch_adj_t<real, true, false, 256>(h, step, lds256);
    } else if (!big) {
        if (want_lj) launch_adj_t<real, false, true, 256>(h, step, lds256);
        else launch_adj_t<real, false, false, 256>(h, step, lds256);
    } else {
        if (want_lj) launch_adj_t<real, false, true, 64>(h, step, lds64);
        else launch_adj_t<real, false, false, 64>(h, step, lds64);
    }
    return hipGetLastError();
}

hipError_t launch_pair_adjoint(irbe_ctx* h, uint64_t step, bool want_q, bool want_lj)
{
    (void)want_q;
    hipError_t e = launch_fill_bytes0(h->stream, h->gscat, 3 * (size_t)h->cfg.n_atoms * h->real_size);
    if (e != hipSuccess) return e;
    e = launch_fill_bytes0(h->stream, h->gqscat, (size_t)h->cfg.n_atoms * h->real_size);
    if (e != hipSuccess) return e;
    return h->fp64 ? launch_adj_r<double>(h, step, want_lj) : launch_adj_r<float>(h, step, want_lj);
}

}  // namespace irbe
