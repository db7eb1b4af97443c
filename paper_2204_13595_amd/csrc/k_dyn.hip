// Langevin dynamics with rigid bond constraints, and the observables of the
// water runs (kinetic energy, mean-squared displacement, radial distribution).
//
// Equations of motion: the underdamped Langevin equations used in the paper's
// convergence analysis (Sec. 3), m dv = (F - gamma m v) dt + sqrt(2 gamma m kT) dW,
// integrated by the splitting kick - drift - noise - drift in leapfrog form (one
// force evaluation per step; Algorithm 1 leaves the integrator open), with the
// bond lengths of each group of at most three atoms held fixed. Per group, one
// thread, all in FP64:
//   1. v += h w F                                  (w = 1/m)
//   2. v += w sum_k mu_k g_k                       relative velocity along each
//                                                  constraint vector r_k = x_q - x_p zero
//   3. y = x + h/2 v
//   4. v = a v + sqrt((1 - a^2) kT w) xi           a = exp(-gamma h)
//   5. y += h/2 v
//   6. x' = y + w sum_k lambda_k g_k               |x'_q - x'_p| = d_k (Newton's method)
//   7. v += (x' - y) / h
// g_k moves p by -r_k and q by +r_k. xi: the Philox4x32-10 block of counter
// (atom, 2^31, step low, 2 step high) under the key seed (the shell batch streams
// use blocks below 2^31 and the k draw has tag 1 in the last word), Box-Muller
// on the word pairs (w0, w1) and (w2, w3).
// Nose-Hoover (the thermostat of the paper's water runs, Sec. 4): step 4 is the
// friction of the thermostat variable instead, v = exp(-xi h) v, and after the
// step xi += h (2 K / (n_dof kT) - 1) / tau^2 with K the kinetic energy of the
// new velocities and n_dof = 3 N - (constraints) - 3.
#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "irbe.h"
#include "irbe_device.hpp"

namespace irbe {
namespace {

constexpr int kDynBlock = 256;
constexpr int kPartBlocks = 1024;  // grid of the reductions (grid-stride), one FP64 partial per block
constexpr int kMaxNewton = 50;
constexpr double kConstraintTol = 1e-14;  // |s^2 - d^2| / d^2 at convergence
enum : uint32_t { DYN_NONFINITE = 1u, DYN_NOCONVERGE = 2u, DYN_BADINDEX = 4u };

struct V3 {
    double x, y, z;
};
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Slot pairs of the three constraints and the sign of slot s in constraint k
// (+1 second atom, -1 first atom, 0 not in it).
__device__ __forceinline__ int pair_p(int k) { return k == 2 ? 1 : 0; }
__device__ __forceinline__ int pair_q(int k) { return k == 0 ? 1 : 2; }
__device__ __forceinline__ double sgn(int s, int k) { return s == pair_q(k) ? 1.0 : (s == pair_p(k) ? -1.0 : 0.0); }

// Solves the 3x3 system A x = b by Gaussian elimination with partial pivoting.
__device__ __forceinline__ void solve3(double A[3][3], double b[3], double x[3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (piv != c) {
            for (int t = 0; t < 3; ++t) {
                const double u = A[c][t];
                A[c][t] = A[piv][t];
                A[piv][t] = u;
            }
            const double u = b[c];
            b[c] = b[piv];
            b[piv] = u;
        }
        for (int r = c + 1; r < 3; ++r) {
            const double f = A[r][c] / A[c][c];
            for (int t = c; t < 3; ++t) A[r][t] -= f * A[c][t];
            b[r] -= f * b[c];
        }
    }
    for (int c = 2; c >= 0; --c) {
        double s = b[c];
        for (int t = c + 1; t < 3; ++t) s -= A[c][t] * x[t];
        x[c] = s / A[c][c];
    }
}

__device__ __forceinline__ V3 load3(const double* p, int64_t i) { return {p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }
template <typename real>
__device__ __forceinline__ V3 load3r(const real* p, int64_t i)
{
    return {(double)p[3 * i], (double)p[3 * i + 1], (double)p[3 * i + 2]};
}
__device__ __forceinline__ void store3(double* p, int64_t i, V3 v)
{
    p[3 * i] = v.x;
    p[3 * i + 1] = v.y;
    p[3 * i + 2] = v.z;
}

// Three standard normals of atom i (Box-Muller on the block's word pairs).
__device__ __forceinline__ V3 noise3(uint64_t seed, uint64_t step, int64_t i)
{
    const Words4 w = philox10((uint32_t)i, 0x80000000u, (uint32_t)step, (uint32_t)(step >> 32) << 1,
                              (uint32_t)seed, (uint32_t)(seed >> 32));
    const double scale = 2.3283064365386963e-10;  // 2^-32
    const double r1 = sqrt(-2.0 * log(((double)w.x + 1.0) * scale));
    const double r2 = sqrt(-2.0 * log(((double)w.z + 1.0) * scale));
    const double t1 = 2.0 * 3.14159265358979323846 * ((double)w.y * scale);
    const double t2 = 2.0 * 3.14159265358979323846 * ((double)w.w * scale);
    return {r1 * cos(t1), r1 * sin(t1), r2 * cos(t2)};
}

template <typename real>
__global__ __launch_bounds__(kDynBlock) void k_langevin_step(int64_t n_groups, const int32_t* __restrict__ groups,
                                                             const double* __restrict__ lengths,
                                                             const double* __restrict__ inv_mass, double* pos,
                                                             double* vel, const real* __restrict__ force, double h,
                                                             double a, double kT, uint64_t seed, uint64_t step,
                                                             const double* __restrict__ nh,
                                                             real* __restrict__ pos_copy, uint32_t* err)
{
    const int64_t g = (int64_t)blockIdx.x * kDynBlock + threadIdx.x;
    if (g >= n_groups) return;
    int at[3];
    V3 x[3], v[3], y[3];
    double w[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        at[s] = groups[3 * g + s];
        const bool used = at[s] >= 0;
        const int64_t i = used ? at[s] : 0;
        x[s] = used ? load3(pos, i) : V3{0, 0, 0};
        v[s] = used ? load3(vel, i) : V3{0, 0, 0};
        w[s] = used ? inv_mass[i] : 0.0;
        const V3 f = used ? load3r(force, i) : V3{0, 0, 0};
        v[s] = v[s] + (h * w[s]) * f;  // 1
    }
    bool act[3];
    double d2[3];
    V3 r[3];
    int n_act = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double len = lengths[3 * g + k];
        act[k] = at[pair_p(k)] >= 0 && at[pair_q(k)] >= 0 && len > 0.0;
        d2[k] = act[k] ? len * len : 1.0;
        r[k] = x[pair_q(k)] - x[pair_p(k)];
        n_act += act[k] ? 1 : 0;
    }
    // C[k][j] = w_q(k) sgn(q(k), j) - w_p(k) sgn(p(k), j): how constraint j's multiplier moves pair k
    double C[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C[k][j] = act[j] ? w[pair_q(k)] * sgn(pair_q(k), j) - w[pair_p(k)] * sgn(pair_p(k), j) : 0.0;
    if (n_act > 0) {  // 2
        double M[3][3], b[3], mu[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const V3 vr = v[pair_q(k)] - v[pair_p(k)];
#pragma unroll
            for (int j = 0; j < 3; ++j) M[k][j] = act[k] ? C[k][j] * dot(r[j], r[k]) : (j == k ? 1.0 : 0.0);
            b[k] = act[k] ? -dot(vr, r[k]) : 0.0;
        }
        solve3(M, b, mu);
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (act[j]) v[s] = v[s] + (w[s] * sgn(s, j) * mu[j]) * r[j];
    }
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        y[s] = x[s] + (0.5 * h) * v[s];  // 3
        if (at[s] >= 0) {
            if (nh) {
                v[s] = exp(-nh[0] * h) * v[s];  // 4, Nose-Hoover
            } else {
                const V3 xi = noise3(seed, step, at[s]);
                v[s] = a * v[s] + sqrt((1.0 - a * a) * kT * w[s]) * xi;  // 4
            }
        }
        y[s] = y[s] + (0.5 * h) * v[s];  // 5
    }
    V3 xn[3] = {y[0], y[1], y[2]};
    if (n_act > 0) {  // 6
        double lam[3] = {0.0, 0.0, 0.0};
        bool done = false;
        for (int it = 0; it < kMaxNewton && !done; ++it) {
            V3 sv[3];
            double f[3];
            double worst = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                V3 sk = y[pair_q(k)] - y[pair_p(k)];
#pragma unroll
                for (int j = 0; j < 3; ++j) sk = sk + (C[k][j] * lam[j]) * r[j];
                sv[k] = sk;
                f[k] = act[k] ? dot(sk, sk) - d2[k] : lam[k];
                if (act[k]) worst = fmax(worst, fabs(f[k] / d2[k]));
            }
            if (worst < kConstraintTol) {
                done = true;
                break;
            }
            double J[3][3], dl[3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int j = 0; j < 3; ++j) J[k][j] = act[k] ? 2.0 * C[k][j] * dot(sv[k], r[j]) : (j == k ? 1.0 : 0.0);
            solve3(J, f, dl);
#pragma unroll
            for (int k = 0; k < 3; ++k) lam[k] -= dl[k];
        }
        if (!done) atomicOr(err, DYN_NOCONVERGE);
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (act[j]) xn[s] = xn[s] + (w[s] * sgn(s, j) * lam[j]) * r[j];
    }
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        if (at[s] < 0) continue;
        v[s] = v[s] + (1.0 / h) * (xn[s] - y[s]);  // 7
        if (!(isfinite(xn[s].x) && isfinite(xn[s].y) && isfinite(xn[s].z) && isfinite(v[s].x) &&
              isfinite(v[s].y) && isfinite(v[s].z)))
            atomicOr(err, DYN_NONFINITE);
        store3(pos, at[s], xn[s]);
        store3(vel, at[s], v[s]);
        if (pos_copy) {
            pos_copy[3 * (int64_t)at[s]] = (real)xn[s].x;
            pos_copy[3 * (int64_t)at[s] + 1] = (real)xn[s].y;
            pos_copy[3 * (int64_t)at[s] + 2] = (real)xn[s].z;
        }
    }
}

// Per-block FP64 partial sums (grid-stride over i < n) of sum m |v|^2 / 2
// (KIND 0) or of |pos[sel] - ref[sel]|^2 (KIND 1); a second launch sums the
// kPartBlocks partials in a fixed order.
template <int KIND>
__global__ __launch_bounds__(kDynBlock) void k_sum_partial(int64_t n, const double* __restrict__ a,
                                                           const double* __restrict__ b,
                                                           const int32_t* __restrict__ sel, int64_t n_atoms,
                                                           double* __restrict__ part, uint32_t* err)
{
    __shared__ double red[kDynBlock / 64];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kDynBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kDynBlock) {
        if (KIND == 0) {
            const V3 v = load3(a, i);
            acc += 0.5 * dot(v, v) / b[i];
        } else {
            const int64_t j = sel[i];
            if (j < 0 || j >= n_atoms) {  // a selection outside the system: flagged, not read
                atomicOr(err, DYN_BADINDEX);
                continue;
            }
            const V3 d = load3(a, j) - load3(b, j);
            acc += dot(d, d);
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < kDynBlock / 64; ++t) s += red[t];
        part[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kDynBlock) void k_sum_final(const double* __restrict__ part, double scale,
                                                         double* __restrict__ out)
{
    __shared__ double red[kDynBlock / 64];
    double acc = 0.0;
    for (int t = threadIdx.x; t < kPartBlocks; t += kDynBlock) acc += part[t];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < kDynBlock / 64; ++t) s += red[t];
        out[0] = s * scale;
    }
}

// Nose-Hoover variable after a step: K from the kinetic partials of the new
// velocities, nh[1] += h xi (the integral of xi, for the conserved quantity),
// then xi += h (2 K / (n_dof kT) - 1) / tau^2.
__global__ __launch_bounds__(kDynBlock) void k_nh_update(const double* __restrict__ part, double dof_kT, double h,
                                                         double inv_tau2, double* __restrict__ nh)
{
    __shared__ double red[kDynBlock / 64];
    double acc = 0.0;
    for (int t = threadIdx.x; t < kPartBlocks; t += kDynBlock) acc += part[t];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double K = 0.0;
        for (int t = 0; t < kDynBlock / 64; ++t) K += red[t];
        const double xi = nh[0];
        nh[1] += h * xi;
        nh[0] = xi + h * (2.0 * K / dof_kT - 1.0) * inv_tau2;
    }
}

__global__ void k_copy2(const double* __restrict__ a, double* __restrict__ b)
{
    if (threadIdx.x < 2) b[threadIdx.x] = a[threadIdx.x];
}

// Pair-distance histogram: pairs a < b of selection A (sel_b == nullptr), or
// every pair of an atom of A and a different atom of B; minimum image per axis,
// FP64 without contraction so that every distance and bin is the plain
// definition's. Block: 256 atoms a, tiles of 256 atoms b staged in LDS; bins
// counted in LDS, then added to the caller's 64-bit histogram.
constexpr int kRdfMaxBins = 8192;

__global__ __launch_bounds__(kDynBlock) void k_rdf(int64_t m, const double* __restrict__ pos, int64_t n_atoms,
                                                   const int32_t* __restrict__ sel, int64_t mb,
                                                   const int32_t* __restrict__ sel_b, double box, double r_max,
                                                   double width, int n_bins, unsigned long long* __restrict__ hist,
                                                   uint32_t* err)
{
#pragma clang fp contract(off)
    __shared__ uint32_t bins[kRdfMaxBins];
    __shared__ V3 tile[kDynBlock];
    for (int t = threadIdx.x; t < n_bins; t += kDynBlock) bins[t] = 0u;
    __shared__ int32_t tile_id[kDynBlock];
    const bool cross = sel_b != nullptr;
    const int32_t* sb = cross ? sel_b : sel;
    const int64_t nb = cross ? mb : m;
    const int64_t a0 = (int64_t)blockIdx.x * kDynBlock;
    const int64_t a = a0 + threadIdx.x;
    // selections outside the system are flagged and their atoms skipped (never read)
    int32_t ia = a < m ? sel[a] : -1;
    if (a < m && (ia < 0 || ia >= n_atoms)) {
        atomicOr(err, DYN_BADINDEX);
        ia = -1;
    }
    const bool a_ok = ia >= 0;
    const V3 pa = a_ok ? load3(pos, ia) : V3{0, 0, 0};
    for (int64_t b0 = cross ? 0 : a0; b0 < nb; b0 += kDynBlock) {
        __syncthreads();
        if (b0 + threadIdx.x < nb) {
            int32_t ib = sb[b0 + threadIdx.x];
            if (ib < 0 || ib >= n_atoms) {
                atomicOr(err, DYN_BADINDEX);
                ib = -1;
            }
            tile_id[threadIdx.x] = ib;
            tile[threadIdx.x] = ib >= 0 ? load3(pos, ib) : V3{0, 0, 0};
        }
        __syncthreads();
        const int cnt = (int)min<int64_t>(kDynBlock, nb - b0);
        if (a_ok)
            for (int t = 0; t < cnt; ++t) {
                if (tile_id[t] < 0 || (cross ? tile_id[t] == ia : b0 + t <= a)) continue;
                V3 d = tile[t] - pa;
                d.x = d.x - box * rint(d.x / box);
                d.y = d.y - box * rint(d.y / box);
                d.z = d.z - box * rint(d.z / box);
                const double r = sqrt(d.x * d.x + d.y * d.y + d.z * d.z);
                if (r < r_max) atomicAdd(&bins[min((int)floor(r / width), n_bins - 1)], 1u);
            }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n_bins; t += kDynBlock)
        if (bins[t]) atomicAdd(&hist[t], (unsigned long long)bins[t]);
}

__global__ void k_clear_word(uint32_t* w) { *w = 0u; }

int64_t nblocks(int64_t n) { return (n + kDynBlock - 1) / kDynBlock; }

thread_local std::string g_dyn_create_error;

}  // namespace
}  // namespace irbe

using namespace irbe;

struct irbe_dyn_ctx {
    irbe_dyn_config cfg{};
    hipStream_t stream = nullptr;
    std::string last_error;
    bool have_system = false;
    int32_t* groups = nullptr;  // [G][3]
    double* lengths = nullptr;  // [G][3]
    double* inv_mass = nullptr; // [N]
    double* part = nullptr;     // [kPartBlocks]
    uint32_t* err = nullptr;
    double* nh = nullptr;       // Nose-Hoover {xi, integral of xi dt}
    int64_t n_dof = 0;          // 3 N - (constraints) - 3
};

namespace {

irbe_status dyn_fail(irbe_dyn_ctx* d, irbe_status st, const std::string& msg)
{
    if (d) d->last_error = msg;
    else g_dyn_create_error = msg;
    return st;
}

irbe_status dyn_hip(irbe_dyn_ctx* d, hipError_t e, const char* where)
{
    return dyn_fail(d, e == hipErrorOutOfMemory ? IRBE_ENOMEM : IRBE_EHIP, std::string(where) + ": " +
                                                                              hipGetErrorString(e));
}

#define DYN_TRY(d, expr, where)                            \
    do {                                                   \
        const hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return dyn_hip(d, e_, where); \
    } while (0)

void dyn_free(irbe_dyn_ctx* d)
{
    for (void* p : {(void*)d->groups, (void*)d->lengths, (void*)d->inv_mass, (void*)d->part, (void*)d->err,
                    (void*)d->nh})
        if (p) (void)hipFree(p);
    delete d;
}

}  // namespace

extern "C" {

irbe_status irbe_dyn_create(const irbe_dyn_config* cfg, void* hip_stream, irbe_dyn_handle* out)
{
    if (!cfg || !out) return dyn_fail(nullptr, IRBE_EINVAL, "null argument");
    *out = nullptr;
    const irbe_dyn_config& c = *cfg;
    if (c.abi_version != IRBE_ABI_VERSION) return dyn_fail(nullptr, IRBE_EINVAL, "abi_version mismatch");
    if (c.force_precision != IRBE_MIXED_FP32 && c.force_precision != IRBE_FP64)
        return dyn_fail(nullptr, IRBE_EINVAL, "bad force_precision");
    if (c.n_atoms < 1 || c.n_atoms > (int64_t(1) << 31) - 1) return dyn_fail(nullptr, IRBE_EINVAL, "n_atoms out of range");
    if (c.n_groups < 1 || c.n_groups > c.n_atoms) return dyn_fail(nullptr, IRBE_EINVAL, "need 1 <= n_groups <= n_atoms");
    if (!(c.dt > 0.0) || !std::isfinite(c.dt)) return dyn_fail(nullptr, IRBE_EINVAL, "need dt > 0");
    if (!(c.gamma >= 0.0) || !std::isfinite(c.gamma)) return dyn_fail(nullptr, IRBE_EINVAL, "need gamma >= 0");
    if (!(c.kT >= 0.0) || !std::isfinite(c.kT)) return dyn_fail(nullptr, IRBE_EINVAL, "need kT >= 0");
    if (c.thermostat != IRBE_LANGEVIN && c.thermostat != IRBE_NOSE_HOOVER)
        return dyn_fail(nullptr, IRBE_EINVAL, "bad thermostat");
    if (c.thermostat == IRBE_NOSE_HOOVER && (!(c.tau > 0.0) || !std::isfinite(c.tau) || !(c.kT > 0.0)))
        return dyn_fail(nullptr, IRBE_EINVAL, "Nose-Hoover needs tau > 0 and kT > 0");
    irbe_dyn_ctx* d = new (std::nothrow) irbe_dyn_ctx();
    if (!d) return dyn_fail(nullptr, IRBE_ENOMEM, "host allocation failed");
    d->cfg = c;
    d->stream = (hipStream_t)hip_stream;
    hipError_t e = hipMalloc((void**)&d->groups, 3 * sizeof(int32_t) * (size_t)c.n_groups);
    if (e == hipSuccess) e = hipMalloc((void**)&d->lengths, 3 * sizeof(double) * (size_t)c.n_groups);
    if (e == hipSuccess) e = hipMalloc((void**)&d->inv_mass, sizeof(double) * (size_t)c.n_atoms);
    if (e == hipSuccess) e = hipMalloc((void**)&d->part, sizeof(double) * kPartBlocks);
    if (e == hipSuccess) e = hipMalloc((void**)&d->err, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&d->nh, 2 * sizeof(double));
    if (e == hipSuccess) {
        const double zero[2] = {0.0, 0.0};
        e = hipMemcpyAsync(d->nh, zero, sizeof(zero), hipMemcpyHostToDevice, d->stream);
    }
    if (e == hipSuccess) {
        k_clear_word<<<1, 1, 0, d->stream>>>(d->err);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
    if (e != hipSuccess) {
        dyn_free(d);
        return dyn_fail(nullptr, e == hipErrorOutOfMemory ? IRBE_ENOMEM : IRBE_EHIP,
                        std::string("create: ") + hipGetErrorString(e));
    }
    *out = d;
    return IRBE_OK;
}

irbe_status irbe_dyn_set_system(irbe_dyn_handle d, const double* inv_mass, const int32_t* groups,
                                const double* lengths)
{
    if (!d || !inv_mass || !groups || !lengths) return dyn_fail(d, IRBE_EINVAL, "null argument");
    const int64_t n = d->cfg.n_atoms, G = d->cfg.n_groups;
    std::vector<double> w((size_t)n), len((size_t)(3 * G));
    std::vector<int32_t> gr((size_t)(3 * G));
    DYN_TRY(d, hipMemcpyAsync(w.data(), inv_mass, w.size() * 8, hipMemcpyDeviceToHost, d->stream), "set_system");
    DYN_TRY(d, hipMemcpyAsync(gr.data(), groups, gr.size() * 4, hipMemcpyDeviceToHost, d->stream), "set_system");
    DYN_TRY(d, hipMemcpyAsync(len.data(), lengths, len.size() * 8, hipMemcpyDeviceToHost, d->stream), "set_system");
    DYN_TRY(d, hipStreamSynchronize(d->stream), "set_system");
    std::vector<uint8_t> seen((size_t)n, 0);
    int64_t n_con = 0;
    for (int64_t g = 0; g < G; ++g) {
        static const int pp[3] = {0, 0, 1}, pq[3] = {1, 2, 2};
        for (int k = 0; k < 3; ++k)
            n_con += (gr[3 * g + pp[k]] >= 0 && gr[3 * g + pq[k]] >= 0 && len[3 * g + k] > 0.0) ? 1 : 0;
        if (gr[3 * g] < 0) return dyn_fail(d, IRBE_EINVAL, "a group's first slot is empty");
        for (int s = 0; s < 3; ++s) {
            const int32_t a = gr[3 * g + s];
            if (a < -1 || a >= n) return dyn_fail(d, IRBE_EINVAL, "group atom index out of range");
            if (a >= 0) {
                if (seen[a]) return dyn_fail(d, IRBE_EINVAL, "an atom is in more than one group slot");
                seen[a] = 1;
            }
            const double l = len[3 * g + s];
            if (!(l >= 0.0) || !std::isfinite(l)) return dyn_fail(d, IRBE_EINVAL, "bad constraint length");
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        if (!seen[i]) return dyn_fail(d, IRBE_EINVAL, "an atom is in no group");
        if (!(w[i] > 0.0) || !std::isfinite(w[i])) return dyn_fail(d, IRBE_EINVAL, "inverse masses must be > 0");
    }
    DYN_TRY(d, hipMemcpyAsync(d->inv_mass, w.data(), w.size() * 8, hipMemcpyHostToDevice, d->stream), "set_system");
    DYN_TRY(d, hipMemcpyAsync(d->groups, gr.data(), gr.size() * 4, hipMemcpyHostToDevice, d->stream), "set_system");
    DYN_TRY(d, hipMemcpyAsync(d->lengths, len.data(), len.size() * 8, hipMemcpyHostToDevice, d->stream), "set_system");
    DYN_TRY(d, hipStreamSynchronize(d->stream), "set_system");
    d->n_dof = 3 * n - n_con - 3;
    if (d->cfg.thermostat == IRBE_NOSE_HOOVER && d->n_dof < 1)
        return dyn_fail(d, IRBE_EINVAL, "Nose-Hoover needs at least one degree of freedom");
    d->have_system = true;
    return IRBE_OK;
}

irbe_status irbe_dyn_step(irbe_dyn_handle d, double* pos, double* vel, const void* force, uint64_t step,
                          void* pos_copy)
{
    if (!d || !pos || !vel || !force) return dyn_fail(d, IRBE_EINVAL, "null argument");
    if (!d->have_system) return dyn_fail(d, IRBE_ESTATE, "set_system first");
    const irbe_dyn_config& c = d->cfg;
    const double a = std::exp(-c.gamma * c.dt);
    const unsigned nb = (unsigned)nblocks(c.n_groups);
    const bool nose = c.thermostat == IRBE_NOSE_HOOVER;
    const double* nh = nose ? d->nh : nullptr;
    if (c.force_precision == IRBE_FP64)
        k_langevin_step<double><<<nb, kDynBlock, 0, d->stream>>>(c.n_groups, d->groups, d->lengths, d->inv_mass, pos,
                                                                 vel, (const double*)force, c.dt, a, c.kT, c.seed,
                                                                 step, nh, (double*)pos_copy, d->err);
    else
        k_langevin_step<float><<<nb, kDynBlock, 0, d->stream>>>(c.n_groups, d->groups, d->lengths, d->inv_mass, pos,
                                                                vel, (const float*)force, c.dt, a, c.kT, c.seed, step,
                                                                nh, (float*)pos_copy, d->err);
    DYN_TRY(d, hipGetLastError(), "step");
    if (nose) {
        k_sum_partial<0><<<kPartBlocks, kDynBlock, 0, d->stream>>>(c.n_atoms, vel, d->inv_mass, nullptr, c.n_atoms,
                                                                   d->part, d->err);
        DYN_TRY(d, hipGetLastError(), "step");
        k_nh_update<<<1, kDynBlock, 0, d->stream>>>(d->part, (double)d->n_dof * c.kT, c.dt, 1.0 / (c.tau * c.tau),
                                                    d->nh);
        DYN_TRY(d, hipGetLastError(), "step");
    }
    return IRBE_OK;
}

irbe_status irbe_dyn_kinetic(irbe_dyn_handle d, const double* vel, double* out)
{
    if (!d || !vel || !out) return dyn_fail(d, IRBE_EINVAL, "null argument");
    if (!d->have_system) return dyn_fail(d, IRBE_ESTATE, "set_system first");
    k_sum_partial<0><<<kPartBlocks, kDynBlock, 0, d->stream>>>(d->cfg.n_atoms, vel, d->inv_mass, nullptr,
                                                               d->cfg.n_atoms, d->part, d->err);
    DYN_TRY(d, hipGetLastError(), "kinetic");
    k_sum_final<<<1, kDynBlock, 0, d->stream>>>(d->part, 1.0, out);
    DYN_TRY(d, hipGetLastError(), "kinetic");
    return IRBE_OK;
}

irbe_status irbe_dyn_msd(irbe_dyn_handle d, const double* pos, const double* ref, const int32_t* sel, int64_t m,
                         double* out)
{
    if (!d || !pos || !ref || !sel || !out) return dyn_fail(d, IRBE_EINVAL, "null argument");
    if (m < 1 || m > d->cfg.n_atoms) return dyn_fail(d, IRBE_EINVAL, "need 1 <= m <= n_atoms");
    k_sum_partial<1><<<kPartBlocks, kDynBlock, 0, d->stream>>>(m, pos, ref, sel, d->cfg.n_atoms, d->part, d->err);
    DYN_TRY(d, hipGetLastError(), "msd");
    k_sum_final<<<1, kDynBlock, 0, d->stream>>>(d->part, 1.0 / (double)m, out);
    DYN_TRY(d, hipGetLastError(), "msd");
    return IRBE_OK;
}

irbe_status irbe_dyn_rdf(irbe_dyn_handle d, const double* pos, const int32_t* sel, int64_t m, const int32_t* sel_b,
                         int64_t m_b, double box, double r_max, int32_t n_bins, uint64_t* hist)
{
    if (!d || !pos || !sel || !hist) return dyn_fail(d, IRBE_EINVAL, "null argument");
    if (m < 0 || m > d->cfg.n_atoms) return dyn_fail(d, IRBE_EINVAL, "need 0 <= m <= n_atoms");
    if (sel_b && (m_b < 0 || m_b > d->cfg.n_atoms)) return dyn_fail(d, IRBE_EINVAL, "need 0 <= m_b <= n_atoms");
    if (n_bins < 1 || n_bins > kRdfMaxBins) return dyn_fail(d, IRBE_EINVAL, "need 1 <= n_bins <= 8192");
    if (!(box > 0.0) || !(r_max > 0.0) || !std::isfinite(box) || !std::isfinite(r_max))
        return dyn_fail(d, IRBE_EINVAL, "need box > 0 and r_max > 0");
    if (m < 1 || (!sel_b && m < 2) || (sel_b && m_b < 1)) return IRBE_OK;
    k_rdf<<<(unsigned)nblocks(m), kDynBlock, 0, d->stream>>>(m, pos, d->cfg.n_atoms, sel, sel_b ? m_b : 0, sel_b, box,
                                                             r_max, r_max / n_bins, n_bins,
                                                             (unsigned long long*)hist, d->err);
    DYN_TRY(d, hipGetLastError(), "rdf");
    return IRBE_OK;
}

irbe_status irbe_dyn_thermostat_state(irbe_dyn_handle d, double* out)
{
    if (!d || !out) return dyn_fail(d, IRBE_EINVAL, "null argument");
    k_copy2<<<1, 64, 0, d->stream>>>(d->nh, out);
    DYN_TRY(d, hipGetLastError(), "thermostat_state");
    return IRBE_OK;
}

int64_t irbe_dyn_degrees_of_freedom(irbe_dyn_handle d) { return d && d->have_system ? d->n_dof : -1; }

irbe_status irbe_dyn_check(irbe_dyn_handle d)
{
    if (!d) return dyn_fail(d, IRBE_EINVAL, "null argument");
    uint32_t err = 0;
    DYN_TRY(d, hipMemcpyAsync(&err, d->err, sizeof(err), hipMemcpyDeviceToHost, d->stream), "check");
    DYN_TRY(d, hipStreamSynchronize(d->stream), "check");
    if (err) {
        k_clear_word<<<1, 1, 0, d->stream>>>(d->err);
        DYN_TRY(d, hipGetLastError(), "check");
        if (err & DYN_BADINDEX) return dyn_fail(d, IRBE_EINVAL, "an atom selection outside [0, n_atoms)");
        if (err & DYN_NONFINITE) return dyn_fail(d, IRBE_ENONFINITE, "non-finite position or velocity");
        return dyn_fail(d, IRBE_ECONVERGENCE, "constraint iteration did not converge");
    }
    return IRBE_OK;
}

const char* irbe_dyn_last_error(irbe_dyn_handle d)
{
    return d ? d->last_error.c_str() : g_dyn_create_error.c_str();
}

irbe_status irbe_dyn_destroy(irbe_dyn_handle d)
{
    if (!d) return IRBE_OK;
    (void)hipStreamSynchronize(d->stream);
    dyn_free(d);
    return IRBE_OK;
}

}  // extern "C"
