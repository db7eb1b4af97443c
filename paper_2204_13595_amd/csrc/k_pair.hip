// Short-range part of the force (Sec. 2.3) and its adjoint.
//
// Forward, per atom i (cell order), Eqs. (2.10)-(2.12):
//   F_i = sum_{j in C(i)} f_ij + w_i sum_{j in B(i)} f_ij + F_i^excl
// with B(i) a batch of p_shell ranks of S(i) drawn without replacement by
// Floyd's algorithm from the Philox word stream of (seed, step, caller id of
// i), w_i = N_S / p_shell (all members and w_i = 1 when N_S <= p_shell). The
// per-block FP64 sums of the uncorrected short-range force give F^corr.
// Full-list mode: one list of every pair within r_shell, weight 1.
// Stencil sampling (STENCIL): the ranks are drawn from K(i), the atoms of the
// shell stencil's cells (N_S replaced by |K(i)|), turned into atom indices by
// k_stencil_decode, and a drawn atom contributes only when it lies in the
// shell annulus T_c < D^2 <= T_s at the current positions (i itself and i's
// molecule come out of the decode as -1).
// Lists built with a skin (skin): every list entry is tested at the current
// positions, core entries counting only at D^2 <= T_c, shell entries only at
// T_c < D^2 <= T_s and full-list entries only at D^2 <= T_s.
#include <algorithm>
#include <type_traits>

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

// Position (type in .w) and charge of sorted atom j. FP32 evaluations read one
// 16-byte record: the fixed-point coordinates and, in the fourth word, the
// charge rounded to 19 mantissa bits (relative change below 2^-20) with the
// atom's type in the 4 bits this frees, so that a pair costs one gather
// instead of two; FP64 evaluations read the position and the exact charge.
template <typename real>
struct Atoms {
    const uint4* __restrict__ spos;
    const real* __restrict__ sqr;
    const uint4* __restrict__ spq;
    __device__ __forceinline__ void get(int64_t j, uint4& p, real& q) const
    {
        if constexpr (std::is_same<real, float>::value) {
            const uint4 r = spq[j];
            p = make_uint4(r.x, r.y, r.z, r.w & 15u);
            q = __uint_as_float(r.w & ~15u);
        } else {
            p = spos[j];
            q = sqr[j];
        }
    }
};

// Exact squared separation in quanta (minimum image through 32-bit wrap-around).
__device__ __forceinline__ uint64_t dist2_q(uint4 a, uint4 b)
{
    const int32_t dx = (int32_t)(b.x - a.x);
    const int32_t dy = (int32_t)(b.y - a.y);
    const int32_t dz = (int32_t)(b.z - a.z);
    return (uint64_t)((int64_t)dx * dx) + (uint64_t)((int64_t)dy * dy) + (uint64_t)((int64_t)dz * dz);
}

// The shell-membership test on exact squared separations in quanta
// (T_c < D^2 <= T_s), used by stencil sampling and by lists built with a skin.
__device__ __forceinline__ bool in_annulus(uint4 a, uint4 b, uint64_t t_lo, uint64_t t_hi)
{
    const uint64_t d2 = dist2_q(a, b);
    return d2 > t_lo && d2 <= t_hi;
}

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
    const real ec = M::erfc_ex(br, ex);
    const real rinv2 = rinv * rinv;
    const real r6 = rinv2 * rinv2 * rinv2;
    const bool lj_on = r2 < lj.rc2;
    real phi = -qq * rinv2 * (ec * rinv + pp.cgauss * ex);
    phi -= lj_on ? r6 * rinv2 * (lj.a12 * r6 - lj.b6) : (real)0;
    if (EV) {
        uc = qq * ec * rinv;
        ul = lj_on ? r6 * (lj.c12 * r6 - lj.c6) - lj.esh : (real)0;
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

// Force, energy and virial sums of one list (core or shell batch).
template <typename real>
struct PairSum {
    real fx = 0, fy = 0, fz = 0;
    real uc = 0, ul = 0;
    real v[6] = {0, 0, 0, 0, 0, 0};
};

template <typename real, bool EV>
__device__ __forceinline__ void add_pair(PairSum<real>& a, uint4 si, real qi, uint4 sj, real qj, const LJ<real>& lje,
                                         const PairParams<real>& pp)
{
    real dx, dy, dz;
    separation(si, sj, pp.quantum, dx, dy, dz);
    const real r2 = dx * dx + dy * dy + dz * dz;
    real uc, ul;
    const real phi = pair_phi<real, EV>(r2, qi * qj, lje, pp, uc, ul);
    a.fx += phi * dx;
    a.fy += phi * dy;
    a.fz += phi * dz;
    if (EV) {
        a.uc += uc;
        a.ul += ul;
        a.v[0] += phi * dx * dx; a.v[1] += phi * dy * dy; a.v[2] += phi * dz * dz;
        a.v[3] += phi * dx * dy; a.v[4] += phi * dx * dz; a.v[5] += phi * dy * dz;
    }
}

// One Floyd step: draw r in [0, t], insert r or (if taken) t into the bitmap
// (word w of this thread's bitmap at bits[w * stride]). The words of r and of
// t are read together (one memory round trip per step); either one is then
// updated. Every element inserted before this step is below t, so t's own bit
// is clear.
__device__ __forceinline__ int floyd_step(WordStream& st, uint32_t* bits, int stride, int t)
{
    const int r = (int)st.below((uint32_t)t + 1u);
    const uint32_t wr = bits[(r >> 5) * stride];
    const uint32_t wt = bits[(t >> 5) * stride];
    const bool taken = (wr >> (r & 31)) & 1u;
    const int v = taken ? t : r;
    bits[(v >> 5) * stride] = (taken ? wt : wr) | (1u << (v & 31));
    return v;
}

// Floyd's algorithm for atom k (sorted index) when N_S > p~: p~ ranks of
// [0, N_S) without replacement, from the word stream of its caller id.
__device__ __forceinline__ void floyd_row(int64_t k, int ns, const int32_t* __restrict__ perm, int p_shell,
                                          int p_stride, uint64_t seed, uint64_t step, uint32_t* bits, int stride,
                                          uint16_t* __restrict__ ranks)
{
    const int words = (ns + 31) >> 5;
    for (int t = 0; t < words; ++t) bits[t * stride] = 0u;
    WordStream st(seed, step, (uint32_t)perm[k], kTagShell);
    uint16_t* out = ranks + k * (int64_t)p_stride;
    const int t0 = ns - p_shell;
    int c = 0;
    for (; c + 4 <= p_shell; c += 4) {
        const uint32_t v0 = (uint32_t)floyd_step(st, bits, stride, t0 + c);
        const uint32_t v1 = (uint32_t)floyd_step(st, bits, stride, t0 + c + 1);
        const uint32_t v2 = (uint32_t)floyd_step(st, bits, stride, t0 + c + 2);
        const uint32_t v3 = (uint32_t)floyd_step(st, bits, stride, t0 + c + 3);
        *(uint2*)(out + c) = make_uint2(v0 | (v1 << 16), v2 | (v3 << 16));
    }
    for (; c < p_shell; ++c) out[c] = (uint16_t)floyd_step(st, bits, stride, t0 + c);
}

// The same ranks, four steps at a time, for bitmaps in LDS. The four words of
// one Philox block serve steps c .. c+3. Unless a lane's multiply-shift needs
// its rejection test (low product word below the bound: about one draw in
// 10^7), the four draws r are then known before any bitmap access, and their
// membership tests go to LDS together as test-and-set operations, which return
// each word as it was before their own bit was set: r is taken when its bit was
// already set, or when it equals the t of an earlier step of the four that was
// taken (that t is inserted only after the four). A free r is inserted by its
// own test-and-set. From the first block in which some lane of the wavefront
// needs the rejection test, and for the steps after the last full block, the
// one-step form continues with the same word stream.
__device__ __forceinline__ void floyd_row_lds(int64_t k, int ns, const int32_t* __restrict__ perm, int p_shell,
                                              int p_stride, uint64_t seed, uint64_t step, uint32_t* bits, int stride,
                                              uint16_t* __restrict__ ranks)
{
    const int words = (ns + 31) >> 5;
    for (int t = 0; t < words; ++t) bits[t * stride] = 0u;
    WordStream st(seed, step, (uint32_t)perm[k], kTagShell);
    uint16_t* out = ranks + k * (int64_t)p_stride;
    const int t0 = ns - p_shell;
    int c = 0;
    for (; c + 4 <= p_shell; c += 4) {
        const Words4 b = philox10(st.c0, st.block, st.c2, st.c3, st.k0, st.k1);
        const uint32_t w[4] = {b.x, b.y, b.z, b.w};
        uint32_t r[4];
        bool hard = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t bound = (uint32_t)(t0 + c + j) + 1u;
            const uint64_t m = (uint64_t)w[j] * bound;
            hard |= (uint32_t)m < bound;
            r[j] = (uint32_t)(m >> 32);
        }
        if (__builtin_amdgcn_ballot_w64(hard) != 0) break;  // this block again, one step at a time
        ++st.block;
        uint32_t old[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            old[j] = __hip_atomic_fetch_or(&bits[(r[j] >> 5) * stride], 1u << (r[j] & 31), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WAVEFRONT);
        uint32_t v[4];
        bool taken[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t t = (uint32_t)(t0 + c + j);
            bool tk = (old[j] >> (r[j] & 31)) & 1u;
#pragma unroll
            for (int i = 0; i < j; ++i) tk |= taken[i] && r[j] == t - (uint32_t)(j - i);
            taken[j] = tk;
            v[j] = tk ? t : r[j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t t = (uint32_t)(t0 + c + j);
            __hip_atomic_fetch_or(&bits[(t >> 5) * stride], taken[j] ? 1u << (t & 31) : 0u, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
        *(uint2*)(out + c) = make_uint2(v[0] | (v[1] << 16), v[2] | (v[3] << 16));
    }
    for (; c < p_shell; ++c) out[c] = (uint16_t)floyd_step(st, bits, stride, t0 + c);
}

// ---------------------------------------------------------------------------
// Forward, cooperative form: the shell batch ranks are drawn first (one thread
// per atom, Floyd's algorithm into a row of 16-bit ranks), then one wavefront
// evaluates one atom at a time with its lanes spread over the atom's core
// list, its batch and its excluded pairs. Each atom's list rows are then read
// by one wavefront at one time (coalesced for the core and full lists, one
// short burst of lines for the sampled shell ranks) instead of entry by entry
// over the whole kernel.
// ---------------------------------------------------------------------------
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_draw_batches(int64_t n, const int32_t* __restrict__ perm,
                                                        const int32_t* __restrict__ nshell, int p_shell, int p_stride,
                                                        uint64_t seed, uint64_t step, uint16_t* __restrict__ ranks)
{
    extern __shared__ uint32_t bitmap[];
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= n) return;
    const int ns = nshell[k];
    if (ns <= p_shell) return;
    floyd_row_lds(k, ns, perm, p_shell, p_stride, seed, step, bitmap + threadIdx.x, BLOCK, ranks);
}

// The same with the bitmaps in device memory, for lists too long for LDS: a
// grid of `threads` threads takes the atoms in turn, thread t's bitmap word w
// at bits[w * threads + t].
__global__ __launch_bounds__(256) void k_draw_batches_global(int64_t n, const int32_t* __restrict__ perm,
                                                             const int32_t* __restrict__ nshell, int p_shell,
                                                             int p_stride, uint64_t seed, uint64_t step,
                                                             uint32_t* __restrict__ bits, int threads,
                                                             uint16_t* __restrict__ ranks)
{
    const int t = (int)(blockIdx.x * 256 + threadIdx.x);
    if (t >= threads) return;
    for (int64_t k = t; k < n; k += threads) {
        const int ns = nshell[k];
        if (ns > p_shell) floyd_row(k, ns, perm, p_shell, p_stride, seed, step, bits + t, threads, ranks);
    }
}

// Stencil sampling: K(i), the atoms of the shell stencil's cells around atom
// i's cell at the build, runs over the stencil rows (dz, dy) in order, each row
// being the cells cx + lo .. cx + lo + span - 1 (cyclic), i.e. at most two
// index ranges of the cell-sorted atoms. A wavefront keeps the rows of one cell
// in LDS (one row per lane, prefix sums by wave scan) and turns a rank of K(i)
// into an atom with a binary search over the rows' first ranks.
constexpr int kDecodeRows = 128;  // stencil rows (span^2) supported

template <int ROWS>
struct StencilRows {
    int32_t pre[ROWS];  // first rank of each row
    int32_t a[ROWS];    // first atom of the row's first range
    int32_t la[ROWS];   // length of the first range
    int32_t b[ROWS];    // first atom of the second range (after the wrap)
};

struct StencilArgs {
    const int32_t* cell_start;
    const int32_t* scell;  // cell of each sorted atom at the build
    const int32_t* smol;   // molecule of each sorted atom
    int n_c, lo, span;
};

__device__ __forceinline__ int wrap_cell(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// The rows of build cell `cell` into T (every lane of the wavefront takes part).
template <int ROWS>
__device__ void stencil_rows_build(StencilRows<ROWS>& T, int cell, const StencilArgs& sa, int lane)
{
    const int n_c = sa.n_c, span = sa.span, nrows = span * span;
    const int cx = cell % n_c, cy = (cell / n_c) % n_c, cz = cell / (n_c * n_c);
    const int x0 = wrap_cell(cx + sa.lo, n_c);
    const int la_c = min(span, n_c - x0);  // cells before the wrap
    int base = 0;
    for (int t0 = 0; t0 < nrows; t0 += 64) {
        const int t = t0 + lane;
        int len = 0, va = 0, vla = 0, vb = 0;
        if (t < nrows) {
            const int z = wrap_cell(cz + t / span + sa.lo, n_c);
            const int y = wrap_cell(cy + t % span + sa.lo, n_c);
            const int row = (z * n_c + y) * n_c;
            va = sa.cell_start[row + x0];
            vla = sa.cell_start[row + x0 + la_c] - va;
            vb = sa.cell_start[row];
            len = vla + (span > la_c ? sa.cell_start[row + span - la_c] - vb : 0);
        }
        int incl = len;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        if (t < nrows) {
            T.pre[t] = base + incl - len;
            T.a[t] = va;
            T.la[t] = vla;
            T.b[t] = vb;
        }
        base += __shfl(incl, 63, 64);
    }
}

// Atom (sorted index) of rank r of K(i) for a cell whose rows are in T: the row
// is the last one whose first rank is <= r.
template <int ROWS>
__device__ __forceinline__ int stencil_rows_atom(const StencilRows<ROWS>& T, int nrows, int r)
{
    int lo_k = 0, hi_k = nrows - 1;
    while (lo_k < hi_k) {
        const int mid = (lo_k + hi_k + 1) >> 1;
        if (T.pre[mid] <= r) lo_k = mid;
        else hi_k = mid - 1;
    }
    const int o = r - T.pre[lo_k];
    const int la = T.la[lo_k];
    return o < la ? T.a[lo_k] + o : T.b[lo_k] + (o - la);
}

// 16-bit shell entries (ListCode): the stencil rows of one list-build group,
// one row per lane: first atom and length of the row's first index range, and
// the first atom of its second range minus that length (zeros past the last
// row, so that any code reads a defined entry).
__device__ void group_rows_build(int4* T, int grp, const ListCode& lc, int lane)
{
    T[lane] = make_int4(0, 0, 0, 0);
    if (lane < lc.span * lc.span) {
        const int rowid = grp / lc.gpr;
        const int cz = rowid / lc.n_c, cy = rowid - cz * lc.n_c;
        const int x0 = (grp - rowid * lc.gpr) * lc.G;
        const int span_u = min(lc.G, lc.n_c - x0) - 1 + lc.span;  // cells of the union x range
        const int xu0 = wrap_cell(x0 + lc.lo, lc.n_c);
        const int lenA = min(span_u, lc.n_c - xu0);
        const int dz = lane / lc.span;
        const int z = wrap_cell(cz + dz + lc.lo, lc.n_c);
        const int y = wrap_cell(cy + (lane - dz * lc.span) + lc.lo, lc.n_c);
        const int row = (z * lc.n_c + y) * lc.n_c;
        const int a = lc.cell_start[row + xu0];
        const int na = lc.cell_start[row + xu0 + lenA] - a;
        T[lane] = make_int4(a, na, lc.cell_start[row] - na, 0);
    }
    // (the wavefront's own table: its later reads follow these writes in order)
    __builtin_amdgcn_wave_barrier();
}

// Atom (sorted index) of shell entry e through the rows of its group in T,
// clamped to the last atom: codes of a build that reported a too long row range
// (forces from such lists are wrong, as the error says) still read in bounds.
__device__ __forceinline__ int group_rows_atom(const int4* T, int pb, int e, int last)
{
    const int4 r = T[e >> pb];
    const int p = e & ((1 << pb) - 1);
    return (int)min((uint32_t)(p < r.y ? r.x + p : r.z + p), (uint32_t)last);
}

// A drawn atom j of atom a (sorted indices) counts as a shell pair: not a
// itself, not of a's molecule, and in the shell annulus.
__device__ __forceinline__ bool stencil_member(int64_t a, int j, int mi, int mj, uint4 si, uint4 sj, uint64_t t_core,
                                               uint64_t t_shell)
{
    return j >= 0 && j != (int)a && !(mi >= 0 && mj == mi) && in_annulus(si, sj, t_core, t_shell);
}

// Read-back of the decoded batch (the atoms at the drawn ranks, -1 for i itself
// and i's molecule): one wavefront per apw consecutive atoms.
constexpr int kDecodeBlock = 256;

__global__ __launch_bounds__(kDecodeBlock) void k_stencil_decode(int64_t n, int apw, StencilArgs sa,
                                                                 const int32_t* __restrict__ nshell, int p_shell,
                                                                 int p_stride, const uint16_t* __restrict__ ranks,
                                                                 int32_t* __restrict__ batch_j)
{
    __shared__ StencilRows<kDecodeRows> rows[kDecodeBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t a0 = ((int64_t)blockIdx.x * (kDecodeBlock / 64) + wave) * apw;
    const int64_t a1 = min(n, a0 + apw);
    const int nrows = sa.span * sa.span;
    int cur = -1;
    for (int64_t a = a0; a < a1; ++a) {
        const int cell = sa.scell[a];
        if (cell != cur) {
            stencil_rows_build(rows[wave], cell, sa, lane);
            cur = cell;
        }
        const int m = nshell[a];
        const bool sample = m > p_shell;
        const int cnt = sample ? p_shell : m;
        const int mi = sa.smol[a];
        const uint16_t* rrow = ranks + a * (int64_t)p_stride;
        int32_t* out = batch_j + a * (int64_t)p_stride;
        // the lane's first two slots with their loads issued together
        const int q0 = lane < cnt ? (sample ? (int)rrow[lane] : lane) : -1;
        const int q1 = lane + 64 < cnt ? (sample ? (int)rrow[lane + 64] : lane + 64) : -1;
        int j0 = q0 >= 0 ? stencil_rows_atom(rows[wave], nrows, q0) : -1;
        int j1 = q1 >= 0 ? stencil_rows_atom(rows[wave], nrows, q1) : -1;
        const int m0 = sa.smol[max(j0, 0)], m1 = sa.smol[max(j1, 0)];
        if (j0 == (int)a || (mi >= 0 && m0 == mi)) j0 = -1;
        if (j1 == (int)a || (mi >= 0 && m1 == mi)) j1 = -1;
        if (q0 >= 0) out[lane] = j0;
        if (q1 >= 0) out[lane + 64] = j1;
        for (int c = lane + 128; c < cnt; c += 64) {
            int j = stencil_rows_atom(rows[wave], nrows, sample ? (int)rrow[c] : c);
            if (j == (int)a || (mi >= 0 && sa.smol[j] == mi)) j = -1;
            out[c] = j;
        }
    }
}

// 16-bit shell entries: the drawn atoms of the current batch (the list members
// at the drawn ranks) into batch_j, for the adjoint when no forward at this
// step wrote them. One wavefront per apw consecutive atoms, one group's rows
// per wavefront in LDS.
__global__ __launch_bounds__(kDecodeBlock) void k_list_decode(int64_t n, int apw, ListCode lc,
                                                              const uint16_t* __restrict__ shell16, int cap_shell,
                                                              const int32_t* __restrict__ nshell, int p_shell,
                                                              int p_stride, const uint16_t* __restrict__ ranks,
                                                              int32_t* __restrict__ batch_j)
{
    __shared__ int4 gt[kDecodeBlock / 64][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t a0 = ((int64_t)blockIdx.x * (kDecodeBlock / 64) + wave) * apw;
    const int64_t a1 = min(n, a0 + apw);
    // an atom's first two slots: their ranks (or list positions), -1 past the batch
    auto slots = [&](int64_t a, int& q0, int& q1) {
        const int m = nshell[a];
        const bool sample = m > p_shell;
        const int cnt = sample ? p_shell : m;
        const uint16_t* rrow = ranks + a * (int64_t)p_stride;
        q0 = lane < cnt ? (sample ? (int)rrow[lane] : lane) : -1;
        q1 = lane + 64 < cnt ? (sample ? (int)rrow[lane + 64] : lane + 64) : -1;
    };
    int cur = -1;
    int n_q0 = -1, n_q1 = -1;
    if (a0 < a1) slots(a0, n_q0, n_q1);
    for (int64_t a = a0; a < a1; ++a) {
        const int q0 = n_q0, q1 = n_q1;
        const uint16_t* srow = shell16 + a * (int64_t)cap_shell;
        // this atom's entries, then the next atom's ranks (in flight while these decode)
        const int e0 = q0 >= 0 ? (int)srow[q0] : 0;
        const int e1 = q1 >= 0 ? (int)srow[q1] : 0;
        if (a + 1 < a1) slots(a + 1, n_q0, n_q1);
        const int grp = lc.sgroup[a];
        if (grp != cur) {
            group_rows_build(gt[wave], grp, lc, lane);
            cur = grp;
        }
        int32_t* out = batch_j + a * (int64_t)p_stride;
        if (q0 >= 0) out[lane] = group_rows_atom(gt[wave], lc.pb, e0, (int)n - 1);
        if (q1 >= 0) out[lane + 64] = group_rows_atom(gt[wave], lc.pb, e1, (int)n - 1);
        // the rest (batches of more than 128)
        const int m = nshell[a];
        const bool sample = m > p_shell;
        const int cnt = sample ? p_shell : m;
        const uint16_t* rrow = ranks + a * (int64_t)p_stride;
        for (int c = lane + 128; c < cnt; c += 64)
            out[c] = group_rows_atom(gt[wave], lc.pb, srow[sample ? (int)rrow[c] : c], (int)n - 1);
    }
}

template <typename real>
__device__ __forceinline__ real wave_sum_r(real v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

constexpr int kCoopBlock = 256;

// A core pair (ex = false, accumulated into pc) or an excluded pair (ex = true,
// into px) with one code path: the excluded-pair correction -erf(br)/r equals
// the real-space term erfc(br)/r minus the bare 1/r, so its force factor is the
// Coulomb part of phi plus qq / r^3, without LJ. Forces only.
template <typename real>
__device__ __forceinline__ void add_pair_or_excl(PairSum<real>& pc, PairSum<real>& px, uint4 si, real qi, uint4 sj,
                                                 real qj, const LJ<real>& lj, const PairParams<real>& pp, bool ex)
{
    using M = Math<real>;
    real dx, dy, dz;
    separation(si, sj, pp.quantum, dx, dy, dz);
    const real r2 = dx * dx + dy * dy + dz * dz;
    const real qq = qi * qj;
    const real rinv = M::rsqrt_(r2);
    const real r = r2 * rinv;
    const real br = pp.beta * r;
    const real e = M::exp_(-br * br);
    const real ec = M::erfc_ex(br, e);
    const real rinv2 = rinv * rinv;
    const real r6 = rinv2 * rinv2 * rinv2;
    const real coul = -qq * rinv2 * (ec * rinv + pp.cgauss * e);
    const real ljf = r2 < lj.rc2 ? r6 * rinv2 * (lj.a12 * r6 - lj.b6) : (real)0;
    const real phi = ex ? coul + qq * rinv2 * rinv : coul - ljf;
    const real fx = phi * dx, fy = phi * dy, fz = phi * dz;
    pc.fx += ex ? (real)0 : fx;
    pc.fy += ex ? (real)0 : fy;
    pc.fz += ex ? (real)0 : fz;
    px.fx += ex ? fx : (real)0;
    px.fy += ex ? fy : (real)0;
    px.fz += ex ? fz : (real)0;
}

// Excluded-pair correction of one pair, accumulated into px.
template <typename real, bool EV>
__device__ __forceinline__ void add_excl(PairSum<real>& px, uint4 si, real qi, uint4 sj, real qj,
                                         const PairParams<real>& pp)
{
    real dx, dy, dz;
    separation(si, sj, pp.quantum, dx, dy, dz);
    const real r2 = dx * dx + dy * dy + dz * dz;
    real u;
    const real psi = excl_psi<real, EV>(r2, qi * qj, pp, u);
    px.fx += psi * dx;
    px.fy += psi * dy;
    px.fz += psi * dz;
    if (EV) {
        px.uc += u;
        px.v[0] += psi * dx * dx; px.v[1] += psi * dy * dy; px.v[2] += psi * dz * dz;
        px.v[3] += psi * dx * dy; px.v[4] += psi * dx * dz; px.v[5] += psi * dy * dz;
    }
}

template <typename real, bool FULL, bool EV, bool STENCIL, bool SKIN, bool ENC>
__global__ __launch_bounds__(kCoopBlock) void k_pair_coop(
    int64_t n, int apw, PairParams<real> pp, const uint4* __restrict__ spos, const real* __restrict__ sqr,
    const uint4* __restrict__ spq, const int2* __restrict__ sxr, const int32_t* __restrict__ sxidx,
    const int32_t* __restrict__ core, const int32_t* __restrict__ ncore, int cap_core,
    const int32_t* __restrict__ shell, const int32_t* __restrict__ nshell, int cap_shell,
    const LJ<real>* __restrict__ lj_g, int n_types, int p_shell, int p_stride, const uint16_t* __restrict__ ranks,
    StencilArgs sa, uint64_t t_core, uint64_t t_shell, real* __restrict__ fsr, double* __restrict__ part,
    int32_t* __restrict__ bj_out, ListCode lc)
{
    __shared__ LJ<real> lj[256];
    __shared__ double red[kPairPartials * (kCoopBlock / 64)];
    __shared__ StencilRows<STENCIL ? kDecodeRows : 1> srows[kCoopBlock / 64];  // stencil rows of one cell per wave
    __shared__ int4 gtab[ENC ? kCoopBlock / 64 : 1][ENC ? 64 : 1];  // 16-bit entries: one group's rows per wave
    const int nt2 = n_types * n_types;
    for (int t = threadIdx.x; t < nt2; t += kCoopBlock) lj[t] = lj_g[t];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    // the wavefront's index as a wave-uniform value, so that its atoms' indices and
    // row addresses are scalar
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t gw = blk * (kCoopBlock / 64) + wave;
    const int64_t a0 = gw * apw;
    const int64_t a1 = min(n, a0 + apw);
    double fc_sum[3] = {0.0, 0.0, 0.0};
    PairSum<real> ev;  // per-lane energy/virial totals (forces unused)
    const Atoms<real> at{spos, sqr, spq};
    // per-atom headers of the wavefront's atoms, one atom per lane, read once
    const int64_t ah = min(a0 + min(lane, apw - 1), n - 1);
    uint4 h_s;
    real h_q;
    at.get(ah, h_s, h_q);
    const int h_nc = FULL ? 0 : ncore[ah];
    const int h_ns = nshell[ah];
    const int2 h_x = sxr[ah];
    const int h_mol = STENCIL ? sa.smol[ah] : 0;
    const int h_grp = ENC ? lc.sgroup[ah] : 0;
    // shell weight N_S / p~ (1 when every member is taken), one division per lane
    const real h_w = (!FULL && h_ns > p_shell) ? (real)((double)h_ns / (double)p_shell) : (real)1;
    const int nrows = sa.span * sa.span;
    int tcell = -1;  // the cell whose stencil rows sit in srows[wave]
    int tgrp = -1;   // the group whose rows sit in gtab[wave]
    // first-level indices of one atom's first pass: the lane's first core entry,
    // its two batch ranks (or shell positions) and its first excluded partner
    // Without energies the excluded partners follow the core entries in one slot
    // (entries nc .. nc + nx - 1 of the combined list); with energies they keep
    // their own slot.
    constexpr bool kFold = !EV;
    auto first_level = [&](int64_t a, int t, int& jc, int& r0, int& r1, int& jx) {
        const int nc = bcast(h_nc, t);
        const int ns = bcast(h_ns, t);
        const int2 xr = make_int2(bcast(h_x.x, t), bcast(h_x.y, t));
        const bool sample = !FULL && ns > p_shell;
        const int cnt = sample ? p_shell : ns;
        const uint16_t* rrow = ranks + a * (int64_t)p_stride;
        if (kFold)
            jc = lane < nc ? core[a * (int64_t)cap_core + lane]
                           : (lane < nc + xr.y ? sxidx[xr.x + lane - nc] : -1);
        else
            jc = lane < nc ? core[a * (int64_t)cap_core + lane] : -1;
        r0 = lane < cnt ? (sample ? (int)rrow[lane] : lane) : -1;
        r1 = lane + 64 < cnt ? (sample ? (int)rrow[lane + 64] : lane + 64) : -1;
        if (STENCIL) {
            // ranks of K(i) -> atoms, through the rows of the atom's build cell
            const int cell = sa.scell[a];
            if (cell != tcell) {
                stencil_rows_build(srows[wave], cell, sa, lane);
                tcell = cell;
            }
            if (r0 >= 0) r0 = stencil_rows_atom(srows[wave], nrows, r0);
            if (r1 >= 0) r1 = stencil_rows_atom(srows[wave], nrows, r1);
        }
        jx = (!kFold && lane < xr.y) ? sxidx[xr.x + lane] : -1;
    };
    // second level of an atom's first pass: the shell entries at its two ranks as
    // stored (16-bit codes or indices; the atoms themselves with stencil sampling)
    auto second_level = [&](int64_t a, int r0, int r1, int& e0, int& e1) {
        if (STENCIL) {
            e0 = r0;
            e1 = r1;
        } else if (ENC) {
            const uint16_t* s16 = reinterpret_cast<const uint16_t*>(shell) + a * (int64_t)cap_shell;
            e0 = r0 >= 0 ? (int)s16[r0] : -1;
            e1 = r1 >= 0 ? (int)s16[r1] : -1;
        } else {
            const int32_t* s1 = shell + a * (int64_t)cap_shell;
            e0 = r0 >= 0 ? s1[r0] : -1;
            e1 = r1 >= 0 ? s1[r1] : -1;
        }
    };
    // a pipeline over the wavefront's atoms: while atom a's pairs are evaluated,
    // the shell entries of atom a + 1 and the first level of atom a + 2 are loaded
    // (issued after atom a's gathers, so that waiting for those does not wait for
    // them: the vector memory counter is in order)
    int n_jc = -1, n_e0 = -1, n_e1 = -1, n_jx = -1;  // atom a: first level and shell entries
    int m_jc = -1, m_r0 = -1, m_r1 = -1, m_jx = -1;  // atom a + 1: first level
    if (a0 < a1) {
        int r0, r1;
        first_level(a0, 0, n_jc, r0, r1, n_jx);
        second_level(a0, r0, r1, n_e0, n_e1);
        if (a0 + 1 < a1) first_level(a0 + 1, 1, m_jc, m_r0, m_r1, m_jx);
    }
    for (int64_t a = a0; a < a1; ++a) {
        const int t = (int)(a - a0);
        const int jc = n_jc, e0 = n_e0, e1 = n_e1, jx = n_jx;
        if (ENC) {
            const int grp = bcast(h_grp, t);
            if (grp != tgrp) {
                group_rows_build(gtab[wave], grp, lc, lane);
                tgrp = grp;
            }
        }
        const uint4 si = make_uint4(bcast(h_s.x, t), bcast(h_s.y, t), bcast(h_s.z, t),
                                    bcast(h_s.w, t));
        const real qi = bcast(h_q, t) * pp.ke;
        // LJ coefficients of the pair types (32-bit LDS indexing; n_types^2 <= 256)
        const int li = (int)si.w * n_types;
        auto ljof = [&](uint4 sj) -> const LJ<real>& { return lj[(li + (int)sj.w) & 255]; };
        const int nc = bcast(h_nc, t);
        const int ns = bcast(h_ns, t);
        const int2 xr = make_int2(bcast(h_x.x, t), bcast(h_x.y, t));
        const int32_t* crow = core + a * (int64_t)cap_core;
        const int32_t* srow = shell + a * (int64_t)cap_shell;
        const uint16_t* srow16 = reinterpret_cast<const uint16_t*>(shell) + a * (int64_t)cap_shell;
        // shell member at position q of the atom's list
        auto member = [&](int q) -> int {
            return ENC ? group_rows_atom(gtab[wave], lc.pb, srow16[q], (int)n - 1) : srow[q];
        };
        const uint16_t* rrow = ranks + a * (int64_t)p_stride;
        const bool sample = !FULL && ns > p_shell;
        const int cnt = sample ? p_shell : ns;
        const real w = bcast(h_w, t);
        PairSum<real> pc, ps, px;
        const int js0 = ENC ? (e0 >= 0 ? group_rows_atom(gtab[wave], lc.pb, e0, (int)n - 1) : -1) : e0;
        const int js1 = ENC ? (e1 >= 0 ? group_rows_atom(gtab[wave], lc.pb, e1, (int)n - 1) : -1) : e1;
        const int mi = STENCIL ? bcast(h_mol, t) : 0;
        const int mj0 = STENCIL ? sa.smol[max(js0, 0)] : 0;
        const int mj1 = STENCIL ? sa.smol[max(js1, 0)] : 0;
        if (!FULL && bj_out) {
            // the batch atoms, for the backward expected at this step (with stencil
            // sampling -1 for i itself and i's molecule, as k_stencil_decode writes)
            auto bj = [&](int j, int mj) { return STENCIL && (j == (int)a || (mi >= 0 && mj == mi)) ? -1 : j; };
            int32_t* o = bj_out + a * (int64_t)p_stride;
            if (lane < cnt) o[lane] = bj(js0, mj0);
            if (lane + 64 < cnt) o[lane + 64] = bj(js1, mj1);
        }
        // (unused slots load atom 0, so that every position is one 16-byte load)
        uint4 pjc, pj0, pj1, pjx;
        real qjc, qj0, qj1, qjx;
        at.get(max(jc, 0), pjc, qjc);
        at.get(max(js0, 0), pj0, qj0);
        at.get(max(js1, 0), pj1, qj1);
        if (kFold) {
            pjx = pjc;
            qjx = qjc;
        } else {
            at.get(max(jx, 0), pjx, qjx);
        }
        if (a + 1 < a1) {
            n_jc = m_jc;
            n_jx = m_jx;
            second_level(a + 1, m_r0, m_r1, n_e0, n_e1);
            if (a + 2 < a1) first_level(a + 2, t + 2, m_jc, m_r0, m_r1, m_jx);
        }
        // skin: a core entry counts inside r_core, a list shell entry inside the annulus
        // (the whole ball in full-list mode), at these positions
        auto core_ok = [&](uint4 sj) { return !SKIN || dist2_q(si, sj) <= t_core; };
        auto shell_ok = [&](uint4 sj) {
            if (!SKIN) return true;
            const uint64_t d2 = dist2_q(si, sj);
            return d2 <= t_shell && (FULL || d2 > t_core);
        };
        if (kFold) {
            if (jc >= 0 && (lane >= nc || core_ok(pjc))) add_pair_or_excl(pc, px, si, qi, pjc, qjc, ljof(pjc), pp, lane >= nc);
        } else {
            if (jc >= 0 && core_ok(pjc)) add_pair<real, EV>(pc, si, qi, pjc, qjc, ljof(pjc), pp);
            if (jx >= 0) add_excl<real, EV>(px, si, qi, pjx, qjx, pp);
        }
        if (STENCIL ? stencil_member(a, js0, mi, mj0, si, pj0, t_core, t_shell) : (js0 >= 0 && shell_ok(pj0)))
            add_pair<real, EV>(ps, si, qi, pj0, qj0, ljof(pj0), pp);
        if (STENCIL ? stencil_member(a, js1, mi, mj1, si, pj1, t_core, t_shell) : (js1 >= 0 && shell_ok(pj1)))
            add_pair<real, EV>(ps, si, qi, pj1, qj1, ljof(pj1), pp);
        // the rest (long lists and large batches)
        if (kFold) {
            for (int c = lane + 64; c < nc + xr.y; c += 64) {
                const int j = c < nc ? crow[c] : sxidx[xr.x + c - nc];
                uint4 sj;
                real qj;
                at.get(j, sj, qj);
                if (c >= nc || core_ok(sj)) add_pair_or_excl(pc, px, si, qi, sj, qj, ljof(sj), pp, c >= nc);
            }
        } else {
            for (int c = lane + 64; c < nc; c += 64) {
                const int j = crow[c];
                uint4 sj;
                real qj;
                at.get(j, sj, qj);
                if (core_ok(sj)) add_pair<real, EV>(pc, si, qi, sj, qj, ljof(sj), pp);
            }
            for (int c = lane + 64; c < xr.y; c += 64) {
                uint4 sj;
                real qj;
                at.get(sxidx[xr.x + c], sj, qj);
                add_excl<real, EV>(px, si, qi, sj, qj, pp);
            }
        }
        if (STENCIL && cnt > 128) {
            // the next atom's first pass may have put another cell's rows in place
            const int cell = sa.scell[a];
            if (cell != tcell) {
                stencil_rows_build(srows[wave], cell, sa, lane);
                tcell = cell;
            }
        }
        for (int c = lane + 128; c < cnt; c += 64) {
            if (STENCIL) {
                const int j = stencil_rows_atom(srows[wave], nrows, sample ? (int)rrow[c] : c);
                const int mj = sa.smol[j];
                if (bj_out) bj_out[a * (int64_t)p_stride + c] = (j == (int)a || (mi >= 0 && mj == mi)) ? -1 : j;
                uint4 sj;
                real qj;
                at.get(j, sj, qj);
                if (stencil_member(a, j, mi, mj, si, sj, t_core, t_shell))
                    add_pair<real, EV>(ps, si, qi, sj, qj, ljof(sj), pp);
            } else {
                const int j = member(sample ? (int)rrow[c] : c);
                if (!FULL && bj_out) bj_out[a * (int64_t)p_stride + c] = j;
                uint4 sj;
                real qj;
                at.get(j, sj, qj);
                if (shell_ok(sj)) add_pair<real, EV>(ps, si, qi, sj, qj, ljof(sj), pp);
            }
        }
        // one set of sums: the excluded-pair forces cancel pairwise, so the momentum
        // correction may sum them with the rest
        const real fx = wave_sum_r(pc.fx + w * ps.fx + px.fx);
        const real fy = wave_sum_r(pc.fy + w * ps.fy + px.fy);
        const real fz = wave_sum_r(pc.fz + w * ps.fz + px.fz);
        if (lane == 0) {
            fsr[3 * a + 0] = fx;
            fsr[3 * a + 1] = fy;
            fsr[3 * a + 2] = fz;
            fc_sum[0] += (double)fx;
            fc_sum[1] += (double)fy;
            fc_sum[2] += (double)fz;
        }
        if (EV) {
            ev.uc += pc.uc + w * ps.uc;
            ev.ul += pc.ul + w * ps.ul;
            ev.fx += px.uc;  // excluded-pair energy
#pragma unroll
            for (int c = 0; c < 6; ++c) ev.v[c] += pc.v[c] + w * ps.v[c] + px.v[c];
        }
    }
    double vals[kPairPartials];
    vals[0] = fc_sum[0];
    vals[1] = fc_sum[1];
    vals[2] = fc_sum[2];
    if (EV) {
        vals[3] = 0.5 * (double)ev.uc;
        vals[4] = 0.5 * (double)ev.ul;
        vals[5] = 0.5 * (double)ev.fx;
        for (int c = 0; c < 6; ++c) vals[6 + c] = -0.5 * (double)ev.v[c];
    } else {
        for (int c = 3; c < 12; ++c) vals[c] = 0.0;
    }
    for (int c = 12; c < kPairPartials; ++c) vals[c] = 0.0;
    double out;
    block_sum_vec<12, kCoopBlock>(vals, red, threadIdx.x, out);
    if (threadIdx.x < 12) part[blk * (int64_t)kPairPartials + threadIdx.x] = out;
}

// Core entries and batch slots of the first pass of k_pair_thread.
constexpr int kThreadFirst = 12;

// Sparse lists (every atom's core list and batch within a few dozen entries, as
// in the dilute electrolytes): one thread per atom walks its own core list,
// excluded partners and batch, so that no wavefront lane idles on an atom with
// a handful of pairs. Same sums and partials as k_pair_coop (split lists).
template <typename real, bool EV>
__global__ __launch_bounds__(kCoopBlock) void k_pair_thread(
    int64_t n, PairParams<real> pp, const uint4* __restrict__ spos, const real* __restrict__ sqr,
    const uint4* __restrict__ spq, const int2* __restrict__ sxr, const int32_t* __restrict__ sxidx,
    const int32_t* __restrict__ core, const int32_t* __restrict__ ncore, int cap_core,
    const int32_t* __restrict__ shell, const int32_t* __restrict__ nshell, int cap_shell,
    const LJ<real>* __restrict__ lj_g, int n_types, int p_shell, int p_stride, const uint16_t* __restrict__ ranks,
    uint64_t t_core, uint64_t t_shell, bool skin, real* __restrict__ fsr, double* __restrict__ part,
    int32_t* __restrict__ bj_out)
{
    __shared__ LJ<real> lj[256];
    __shared__ double red[kPairPartials * (kCoopBlock / 64)];
    const int nt2 = n_types * n_types;
    for (int t = threadIdx.x; t < nt2; t += kCoopBlock) lj[t] = lj_g[t];
    __syncthreads();
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t a = blk * kCoopBlock + threadIdx.x;
    double vals[kPairPartials];
    for (int c = 0; c < kPairPartials; ++c) vals[c] = 0.0;
    const Atoms<real> at{spos, sqr, spq};
    if (a < n) {
        uint4 si;
        real qi;
        at.get(a, si, qi);
        qi *= pp.ke;
        // LJ coefficients of the pair types (32-bit LDS indexing; n_types^2 <= 256)
        const int li = (int)si.w * n_types;
        auto ljof = [&](uint4 sj) -> const LJ<real>& { return lj[(li + (int)sj.w) & 255]; };
        PairSum<real> pc, ps, px;
        const int nc = ncore[a];
        const int32_t* crow = core + a * (int64_t)cap_core;
        const int ns = nshell[a];
        const bool sample = ns > p_shell;
        const int cnt = sample ? p_shell : ns;
        const int32_t* srow = shell + a * (int64_t)cap_shell;
        const uint16_t* rrow = ranks + a * (int64_t)p_stride;
        // first pass over up to kThreadFirst core entries and batch slots, each
        // level's loads issued together: core indices and batch ranks, then core
        // positions and shell entries, then shell positions
        int jc[kThreadFirst], js[kThreadFirst];
#pragma unroll
        for (int u = 0; u < kThreadFirst; ++u) jc[u] = u < nc ? crow[u] : -1;
#pragma unroll
        for (int u = 0; u < kThreadFirst; ++u) js[u] = u < cnt ? (sample ? (int)rrow[u] : u) : -1;
        uint4 sc[kThreadFirst];
        real qc[kThreadFirst];
#pragma unroll
        for (int u = 0; u < kThreadFirst; ++u) at.get(max(jc[u], 0), sc[u], qc[u]);
#pragma unroll
        for (int u = 0; u < kThreadFirst; ++u) js[u] = js[u] >= 0 ? srow[js[u]] : -1;
        if (bj_out) {
            // the batch atoms, for the backward expected at this step
#pragma unroll
            for (int u = 0; u < kThreadFirst; ++u)
                if (u < cnt) bj_out[a * (int64_t)p_stride + u] = js[u];
        }
        uint4 ss[kThreadFirst];
        real qs[kThreadFirst];
#pragma unroll
        for (int u = 0; u < kThreadFirst; ++u) at.get(max(js[u], 0), ss[u], qs[u]);
#pragma unroll
        for (int u = 0; u < kThreadFirst; ++u)
            if (jc[u] >= 0 && (!skin || dist2_q(si, sc[u]) <= t_core))
                add_pair<real, EV>(pc, si, qi, sc[u], qc[u], ljof(sc[u]), pp);
#pragma unroll
        for (int u = 0; u < kThreadFirst; ++u)
            if (js[u] >= 0 && (!skin || in_annulus(si, ss[u], t_core, t_shell)))
                add_pair<real, EV>(ps, si, qi, ss[u], qs[u], ljof(ss[u]), pp);
        // the rest four entries at a time: their index and position loads go out together
        for (int c0 = kThreadFirst; c0 < nc; c0 += 4) {
            int j[4];
            uint4 sj[4];
            real qj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) j[u] = c0 + u < nc ? crow[c0 + u] : -1;
#pragma unroll
            for (int u = 0; u < 4; ++u) at.get(max(j[u], 0), sj[u], qj[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (j[u] >= 0 && (!skin || dist2_q(si, sj[u]) <= t_core))
                    add_pair<real, EV>(pc, si, qi, sj[u], qj[u], ljof(sj[u]), pp);
        }
        const int2 xr = sxr[a];
        for (int c = 0; c < xr.y; ++c) {
            uint4 sj;
            real qj;
            at.get(sxidx[xr.x + c], sj, qj);
            add_excl<real, EV>(px, si, qi, sj, qj, pp);
        }
        for (int c0 = kThreadFirst; c0 < cnt; c0 += 4) {
            int r[4], j[4];
            uint4 sj[4];
            real qj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) r[u] = c0 + u < cnt ? (sample ? (int)rrow[c0 + u] : c0 + u) : -1;
#pragma unroll
            for (int u = 0; u < 4; ++u) j[u] = r[u] >= 0 ? srow[r[u]] : -1;
            if (bj_out) {
                // the batch atoms, for the backward expected at this step
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (c0 + u < cnt) bj_out[a * (int64_t)p_stride + c0 + u] = j[u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) at.get(max(j[u], 0), sj[u], qj[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (j[u] >= 0 && (!skin || in_annulus(si, sj[u], t_core, t_shell)))
                    add_pair<real, EV>(ps, si, qi, sj[u], qj[u], ljof(sj[u]), pp);
        }
        const real w = sample ? (real)((double)ns / (double)p_shell) : (real)1;
        const real fx = pc.fx + w * ps.fx + px.fx;
        const real fy = pc.fy + w * ps.fy + px.fy;
        const real fz = pc.fz + w * ps.fz + px.fz;
        fsr[3 * a + 0] = fx;
        fsr[3 * a + 1] = fy;
        fsr[3 * a + 2] = fz;
        vals[0] = (double)fx;
        vals[1] = (double)fy;
        vals[2] = (double)fz;
        if (EV) {
            vals[3] = 0.5 * (double)(pc.uc + w * ps.uc);
            vals[4] = 0.5 * (double)(pc.ul + w * ps.ul);
            vals[5] = 0.5 * (double)px.uc;
            for (int c = 0; c < 6; ++c) vals[6 + c] = -0.5 * (double)(pc.v[c] + w * ps.v[c] + px.v[c]);
        }
    }
    double out;
    block_sum_vec<12, kCoopBlock>(vals, red, threadIdx.x, out);
    if (threadIdx.x < 12) part[blk * (int64_t)kPairPartials + threadIdx.x] = out;
}

static StencilArgs stencil_args(const irbe_ctx* h)
{
    StencilArgs sa;
    sa.cell_start = h->cell_start;
    sa.scell = h->scell;
    sa.smol = h->smol;
    sa.n_c = h->geo.n_c;
    sa.lo = h->geo.lo;
    sa.span = h->geo.hi - h->geo.lo + 1;
    return sa;
}

// Stencil sampling: the drawn atoms of the current batch into h->batch_j (for
// read-back; the pair kernels decode the ranks themselves).
hipError_t launch_stencil_decode(irbe_ctx* h)
{
    if (!h->stencil) return hipErrorInvalidValue;
    const StencilArgs sa = stencil_args(h);
    if (sa.span * sa.span > kDecodeRows) return hipErrorInvalidValue;
    const int64_t n = h->cfg.n_atoms;
    const hipError_t e = ensure_batch_atoms(h);
    if (e != hipSuccess) return e;
    const int apw = 16;
    const int64_t waves = blocks_for(n, apw);
    k_stencil_decode<<<(unsigned)blocks_for(waves, kDecodeBlock / 64), kDecodeBlock, 0, h->stream>>>(
        n, apw, sa, h->nshell, h->cfg.p_shell, h->p_stride, h->ranks, h->batch_j);
    return hipGetLastError();
}

// 16-bit shell entries: the drawn atoms of the current ranks into h->batch_j.
static hipError_t launch_list_decode(irbe_ctx* h)
{
    if (!h->shell16) return hipErrorInvalidValue;
    const int64_t n = h->cfg.n_atoms;
    const hipError_t e = ensure_batch_atoms(h);
    if (e != hipSuccess) return e;
    const int apw = 16;
    const int64_t waves = blocks_for(n, apw);
    k_list_decode<<<(unsigned)blocks_for(waves, kDecodeBlock / 64), kDecodeBlock, 0, h->stream>>>(
        n, apw, h->lcode, reinterpret_cast<const uint16_t*>(h->shell), h->cap_shell, h->nshell, h->cfg.p_shell,
        h->p_stride, h->ranks, h->batch_j);
    return hipGetLastError();
}

// Threads per block of the batch draw and the LDS its bitmaps take (one bitmap
// of the longest list per thread); more than 64 KiB means device memory.
static int draw_block(const irbe_ctx* h, size_t* lds)
{
    const int words = (h->shell_bound() + 31) / 32;
    int block = 256;
    while (block > 64 && (size_t)words * block * 4 > 32 * 1024) block /= 2;
    if (block == 64 && (size_t)words * block * 4 > 64 * 1024) block = 32;
    *lds = (size_t)words * block * 4;
    return block;
}

bool draw_bitmaps_in_lds(const irbe_ctx* h)
{
    size_t lds = 0;
    draw_block(h, &lds);
    return lds <= 64 * 1024;
}

// Batch ranks of every atom for `step` (kept until the lists or the step change).
static hipError_t launch_draw(irbe_ctx* h, uint64_t step)
{
    if (h->full_list || (h->ranks_valid && h->ranks_step == step)) return hipSuccess;
    const int64_t n = h->cfg.n_atoms;
    const int words = (h->shell_bound() + 31) / 32;
    size_t lds = 0;
    const int block = draw_block(h, &lds);
    const unsigned nb = (unsigned)blocks_for(n, block);
    if (lds > 64 * 1024) {
        // bitmaps in device memory: as many threads as fit 1 GiB of bitmaps
        const int64_t threads = std::max<int64_t>(256, std::min<int64_t>(n, ((int64_t)1 << 28) / words) / 256 * 256);
        hipError_t e = ensure_draw_bits(h, (size_t)threads * (size_t)words);
        if (e != hipSuccess) return e;
        k_draw_batches_global<<<(unsigned)(threads / 256), 256, 0, h->stream>>>(
            n, h->perm, h->nshell, h->cfg.p_shell, h->p_stride, h->cfg.seed, step, h->draw_bits, (int)threads,
            h->ranks);
    } else if (block == 256)
        k_draw_batches<256><<<nb, 256, lds, h->stream>>>(n, h->perm, h->nshell, h->cfg.p_shell, h->p_stride,
                                                         h->cfg.seed, step, h->ranks);
    else if (block == 128)
        k_draw_batches<128><<<nb, 128, lds, h->stream>>>(n, h->perm, h->nshell, h->cfg.p_shell, h->p_stride,
                                                         h->cfg.seed, step, h->ranks);
    else if (block == 64)
        k_draw_batches<64><<<nb, 64, lds, h->stream>>>(n, h->perm, h->nshell, h->cfg.p_shell, h->p_stride,
                                                       h->cfg.seed, step, h->ranks);
    else
        k_draw_batches<32><<<nb, 32, lds, h->stream>>>(n, h->perm, h->nshell, h->cfg.p_shell, h->p_stride,
                                                       h->cfg.seed, step, h->ranks);
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        h->ranks_valid = true;
        h->ranks_step = step;
        h->batch_j_valid = h->batch_j_fwd = false;
    }
    return e;
}

template <typename real, bool FULL, bool EV, bool STENCIL, bool SKIN, bool ENC = false>
static hipError_t launch_coop_t(irbe_ctx* h, uint64_t step)
{
    const int64_t n = h->cfg.n_atoms;
    PairParams<real> pp;
    pp.quantum = (real)h->geo.quantum;
    pp.beta = (real)h->cfg.ewald_beta;
    pp.cgauss = (real)(2.0 * h->cfg.ewald_beta / 1.7724538509055160273);
    pp.ke = (real)h->cfg.coulomb_k;
    hipError_t e = launch_draw(h, step);
    if (e != hipSuccess) return e;
    // stencil sampling keeps one cell's stencil rows for consecutive atoms: longer
    // runs of atoms per wavefront pay there, shorter ones with list-drawn batches
    const int apw = STENCIL ? kAtomsPerWaveStencil : (FULL ? kAtomsPerWaveList : kAtomsPerWaveSplit);
    const int64_t waves = blocks_for(n, apw);
    const unsigned nb = (unsigned)blocks_for(waves, kCoopBlock / 64);
    if ((int64_t)nb > h->part_blocks) return hipErrorInvalidValue;
    // the batch atoms for the backward, when one followed the last forward (into a
    // buffer that backward allocated: a forward allocates nothing here)
    int32_t* bj_out = (!FULL && h->keep_batch) ? h->batch_j : nullptr;
    k_pair_coop<real, FULL, EV, STENCIL, SKIN, ENC><<<nb, kCoopBlock, 0, h->stream>>>(
        n, apw, pp, h->spos, (const real*)h->sq_r, h->spq, h->sxr, h->sxidx, h->core, h->ncore, h->cap_core,
        h->shell, h->nshell, h->cap_shell, (const LJ<real>*)h->lj, h->cfg.n_types, h->cfg.p_shell, h->p_stride,
        h->ranks, stencil_args(h), h->geo.t_core, h->geo.t_shell, (real*)h->fsr, h->pair_part, bj_out, h->lcode);
    h->pair_nb = nb;
    if (bj_out) h->batch_j_valid = h->batch_j_fwd = true;
    return hipGetLastError();
}

template <typename real, bool EV>
static hipError_t launch_thread_t(irbe_ctx* h, uint64_t step)
{
    const int64_t n = h->cfg.n_atoms;
    PairParams<real> pp;
    pp.quantum = (real)h->geo.quantum;
    pp.beta = (real)h->cfg.ewald_beta;
    pp.cgauss = (real)(2.0 * h->cfg.ewald_beta / 1.7724538509055160273);
    pp.ke = (real)h->cfg.coulomb_k;
    hipError_t e = launch_draw(h, step);
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)blocks_for(n, kCoopBlock);
    if ((int64_t)nb > h->part_blocks) return hipErrorInvalidValue;
    // the batch atoms for the backward, as in launch_coop_t
    int32_t* bj_out = h->keep_batch ? h->batch_j : nullptr;
    k_pair_thread<real, EV><<<nb, kCoopBlock, 0, h->stream>>>(
        n, pp, h->spos, (const real*)h->sq_r, h->spq, h->sxr, h->sxidx, h->core, h->ncore, h->cap_core, h->shell, h->nshell,
        h->cap_shell, (const LJ<real>*)h->lj, h->cfg.n_types, h->cfg.p_shell, h->p_stride, h->ranks, h->geo.t_core,
        h->geo.t_shell, h->geo.skin, (real*)h->fsr, h->pair_part, bj_out);
    h->pair_nb = nb;
    if (bj_out) h->batch_j_valid = h->batch_j_fwd = true;
    return hipGetLastError();
}

// The cooperative kernel for the list mode, energies and skin.
template <typename real, bool SKIN>
static hipError_t launch_coop_s(irbe_ctx* h, uint64_t step, bool ev)
{
    if (h->full_list)
        return ev ? launch_coop_t<real, true, true, false, SKIN>(h, step)
                  : launch_coop_t<real, true, false, false, SKIN>(h, step);
    if (h->stencil)
        return ev ? launch_coop_t<real, false, true, true, SKIN>(h, step)
                  : launch_coop_t<real, false, false, true, SKIN>(h, step);
    if (h->shell16)
        return ev ? launch_coop_t<real, false, true, false, SKIN, true>(h, step)
                  : launch_coop_t<real, false, false, false, SKIN, true>(h, step);
    return ev ? launch_coop_t<real, false, true, false, SKIN>(h, step)
              : launch_coop_t<real, false, false, false, SKIN>(h, step);
}

// Split lists whose longest core list plus batch stays within this many entries
// take the thread-per-atom kernel (32-bit shell entries only: the cooperative
// kernel decodes the 16-bit ones).
constexpr int kSparsePairs = 32;

template <typename real>
static hipError_t launch_coop_r(irbe_ctx* h, uint64_t step, bool ev)
{
    if (!h->full_list && !h->stencil && !h->shell16 &&
        h->max_core + std::min(h->max_shell, h->cfg.p_shell) <= kSparsePairs)
        return ev ? launch_thread_t<real, true>(h, step) : launch_thread_t<real, false>(h, step);
    return h->geo.skin ? launch_coop_s<real, true>(h, step, ev) : launch_coop_s<real, false>(h, step, ev);
}

// Reduce the per-block partials in a fixed order, in two stages: stage 1 sums
// contiguous ranges of blocks into kReduceSlices slices, stage 2 sums the
// slices: ev_pair[0..11] = totals, fcorr = (sum of the uncorrected short-range
// force) / N when rbl.
constexpr int kReduceSlices = 256;

__global__ __launch_bounds__(kReduceBlock) void k_pair_reduce1(int64_t nb, const double* __restrict__ part,
                                                               double* __restrict__ slices)
{
    __shared__ double lds[12 * (kReduceBlock / 64)];
    const int64_t per = (nb + kReduceSlices - 1) / kReduceSlices;
    const int64_t b0 = blockIdx.x * per, b1 = min(nb, b0 + per);
    double vals[12];
    for (int c = 0; c < 12; ++c) vals[c] = 0.0;
    for (int64_t b = b0 + threadIdx.x; b < b1; b += kReduceBlock)
        for (int c = 0; c < 12; ++c) vals[c] += part[b * kPairPartials + c];
    double out;
    block_sum_vec<12, kReduceBlock>(vals, lds, threadIdx.x, out);
    if (threadIdx.x < 12) slices[blockIdx.x * 12 + threadIdx.x] = out;
}

__global__ __launch_bounds__(kReduceBlock) void k_pair_reduce2(const double* __restrict__ slices, int64_t n, int rbl,
                                                               double* __restrict__ ev_pair,
                                                               double* __restrict__ fcorr)
{
    __shared__ double lds[12 * (kReduceBlock / 64)];
    double vals[12];
    for (int c = 0; c < 12; ++c) vals[c] = 0.0;
    for (int b = threadIdx.x; b < kReduceSlices; b += kReduceBlock)
        for (int c = 0; c < 12; ++c) vals[c] += slices[b * 12 + c];
    double out;
    block_sum_vec<12, kReduceBlock>(vals, lds, threadIdx.x, out);
    if (threadIdx.x < 12) ev_pair[threadIdx.x] = out;
    if (threadIdx.x < 3) fcorr[threadIdx.x] = rbl ? out / (double)n : 0.0;
}

hipError_t launch_pair_reduce(irbe_ctx* h)
{
    k_pair_reduce1<<<kReduceSlices, kReduceBlock, 0, h->stream>>>(h->pair_nb, h->pair_part, h->pair_slices);
    k_pair_reduce2<<<1, kReduceBlock, 0, h->stream>>>(h->pair_slices, h->cfg.n_atoms, h->full_list ? 0 : 1,
                                                      h->ev_pair, h->fcorr);
    return hipGetLastError();
}

hipError_t launch_pair_forces(irbe_ctx* h, uint64_t step, bool ev)
{
    const hipError_t e = h->fp64 ? launch_coop_r<double>(h, step, ev) : launch_coop_r<float>(h, step, ev);
    // each forward renews the prediction: a backward after it sets keep_batch again
    h->keep_batch = false;
    h->fwd_pending = true;
    return e;
}

// ---------------------------------------------------------------------------
// Adjoint of the short-range force (vector-Jacobian product with G = dL/dF at
// fixed lists and batches). With f_ij = phi(r) r_ij, J = phi I + (phi'/r) r r^T
// is symmetric and even in r_ij, so for the symmetric sets (C(i), the full list,
// the excluded pairs) the gradient is gathered per atom:
//   dL/dr_i += sum_j J (G'_j - G'_i),  dL/dq_i += sum_j (ke q_j a(r)) r_ij.(G'_j - G'_i)
// where a(r) is the Coulomb factor of phi / (-ke q_i q_j). The sampled shell
// terms are one-sided: dL/dr_i -= w J G'_i and dL/dr_j += w J G'_i, and likewise
// for the charges. G' = G - mean(G) for the pair terms when the momentum
// correction is applied; excluded pairs use G. LJ table gradients are
// accumulated per (t_i, t_j) entry in FP64.
//
// The scatter onto j is a transpose. Device-scope atomics on this chip are
// executed at the memory side, one transaction per lane, so instead each block
// (a run of consecutive cell-ordered atoms, which lie in one or two cell rows)
// stages its records (j, w J G'_i, charge term) in LDS, counts them per
// (source row, destination row) key, reserves one contiguous range per key in
// the destination row's bucket with a single atomic, and writes the records
// there. A second kernel reduces each row's bucket in LDS and adds the row's
// gradients with plain stores. LDS floating-point atomics are several times
// slower than integer ones here, so the row sums are accumulated in 64-bit
// fixed point, scaled by a power of two chosen from the row's largest record
// (bounded above by the largest component any contributing block staged)
// and record count so that no sum can overflow (integer sums are also
// independent of the order). Records that do not fit (a third source row in
// one block, a full bucket, an atom beyond the LDS row window) fall back to
// device atomics, so the result never depends on the capacities.
// ---------------------------------------------------------------------------
template <typename real>
struct PairGrad {
    real phi, dphi_r;   // phi and phi'(r)/r
    real a_coul;        // erfc/r^3 + 2b e^{-b^2 r^2}/(sqrt(pi) r^2): phi_coul = -qq a_coul
    real c_lj;          // 48 s^12/r^14 - 24 s^6/r^8: phi_lj = -eps c_lj
    real dc_dsig;       // d c_lj / d sigma
};

// LJ constants of one type pair for the adjoint (sigma powers folded in).
template <typename real>
struct LJGrad {
    real a48, b24;    // 48 s^12, 24 s^6:   c_lj = (a48 r^-6 - b24) r^-8
    real a672, b192;  // 672 s^12, 192 s^6: d c_lj / dr = (b192 - a672 r^-6) r^-9
    real as, bs;      // 576 s^11, 144 s^5: d c_lj / d sigma = (as r^-6 - bs) r^-8
    real eps, rc2;    // the LJ term acts at r^2 < rc2
};

template <typename real>
__device__ __forceinline__ LJGrad<real> lj_grad_entry(real sig, real eps, real lj_cut)
{
    const real s2 = sig * sig;
    const real s6 = s2 * s2 * s2;
    const real s12 = s6 * s6;
    LJGrad<real> L;
    L.a48 = (real)48 * s12;
    L.b24 = (real)24 * s6;
    L.a672 = (real)672 * s12;
    L.b192 = (real)192 * s6;
    L.as = sig != (real)0 ? (real)576 * s12 / sig : (real)0;
    L.bs = sig != (real)0 ? (real)144 * s6 / sig : (real)0;
    L.eps = eps;
    L.rc2 = lj_cut > (real)0 ? lj_cut * sig * lj_cut * sig : Math<real>::max_();
    return L;
}

// xp: an excluded pair, whose correction -erf(br)/r is the real-space term
// erfc(br)/r minus the bare 1/r: the Coulomb factor gains -1/r^3, phi gains
// qq/r^3, phi'/r gains -3 qq/r^5, and there is no LJ term.
template <typename real>
__device__ __forceinline__ PairGrad<real> pair_grad(real r2, real qq, const LJGrad<real>& L, const PairParams<real>& pp,
                                                    bool xp = false)
{
    using M = Math<real>;
    const real rinv = M::rsqrt_(r2);
    const real r = r2 * rinv;
    const real br = pp.beta * r;
    const real ex = M::exp_(-br * br);
    const real ec = M::erfc_ex(br, ex);
    const real rinv2 = rinv * rinv;
    const real rinv3 = rinv2 * rinv;
    const real A = ec * rinv3;
    const real B = pp.cgauss * ex * rinv2;
    const real dA = -rinv * (B + (real)3 * A);
    const real dB = -B * ((real)2 * pp.beta * pp.beta * r + (real)2 * rinv);
    const real r6 = rinv2 * rinv2 * rinv2;
    const real r8 = r6 * rinv2;
    const real on = (xp || !(r2 < L.rc2)) ? (real)0 : (real)1;
    const real C = on * r8 * (L.a48 * r6 - L.b24);
    const real dC = on * rinv * r8 * (L.b192 - L.a672 * r6);
    const real eps = on * L.eps;
    PairGrad<real> g;
    g.a_coul = xp ? A + B - rinv3 : A + B;
    g.phi = -qq * g.a_coul - eps * C;
    g.dphi_r = (-qq * (dA + dB) - eps * dC) * rinv - (xp ? (real)3 * qq * rinv2 * rinv3 : (real)0);
    g.c_lj = C;
    g.dc_dsig = on * r8 * (L.as * r6 - L.bs);
    return g;
}

template <typename real>
__device__ __forceinline__ void load3(const real* p, int64_t k, real& x, real& y, real& z)
{
    x = p[3 * k];
    y = p[3 * k + 1];
    z = p[3 * k + 2];
}

// Geometry of the shell-adjoint buckets. Row R = cz n_c + cy holds the atoms of
// cells [R n_c, (R + 1) n_c); its bucket starts at
// floor(cell_start[R n_c] p9 / 8) + kBucketSlack R records (9/8 of the expected
// p_eff records per atom, plus slack).
struct BucketArgs {
    int n_c, lo, span;            // shell stencil offsets lo .. lo + span - 1 per axis
    int64_t p9;                   // 9 * p_eff
    const int32_t* cell_start;
    unsigned long long* cursor;   // [n_c^2] records reserved per destination row
    unsigned long long* rowmax;   // [n_c^2] bits of the largest |record component| (as a non-negative double)
    void* rec_c;                  // real[4 * total]
    uint16_t* rec_j;              // [total]
    unsigned long long* n_atomic; // records that took device atomics instead of a bucket
    const int32_t* brow;          // cell (z, y) at the build of each sorted atom (z << 16 | y), used for the keys
                                  // when positions may have moved since (lists with a skin); null: from positions
};

__device__ __forceinline__ int64_t bucket_start(const BucketArgs& bk, int row)
{
    const int64_t a = bk.cell_start[(int64_t)row * bk.n_c];
    return ((a * bk.p9) >> 3) + (int64_t)kBucketSlack * row;
}

__device__ __forceinline__ int cell_row(uint4 s, int n_c)
{
    const int cz = (int)(((uint64_t)s.z * (uint32_t)n_c) >> 32);
    const int cy = (int)(((uint64_t)s.y * (uint32_t)n_c) >> 32);
    return cz * n_c + cy;
}

// Cell coordinates (z, y) of sorted atom k for the bucket keys: those of its
// cell at the list build when the positions may have moved since, else those
// of its position.
__device__ __forceinline__ void key_cell(const BucketArgs& bk, int64_t k, uint4 s, int& z, int& y)
{
    if (bk.brow) {
        const int b = bk.brow[k];
        z = b >> 16;
        y = b & 0xffff;
    } else {
        z = (int)(((uint64_t)s.z * (uint32_t)bk.n_c) >> 32);
        y = (int)(((uint64_t)s.y * (uint32_t)bk.n_c) >> 32);
    }
}

// Offset d = c_j - c_i of a stencil cell mapped into [lo, lo + span).
__device__ __forceinline__ int stencil_offset(int cj, int ci, int lo, int span, int n_c)
{
    int d = cj - ci;
    if (d < lo) d += n_c;
    if (d >= lo + span) d -= n_c;
    return d;
}

template <typename real>
__device__ __forceinline__ void scatter_atomic(real* gscat, real* gqscat, int64_t j, real x, real y, real z, real q)
{
    atomicAdd(&gscat[3 * j + 0], x);
    atomicAdd(&gscat[3 * j + 1], y);
    atomicAdd(&gscat[3 * j + 2], z);
    atomicAdd(&gqscat[j], q);
}

// One wavefront per atom (cell order), lanes over the atom's lists. BK: the
// shell scatter goes through the LDS-staged buckets (dynamic LDS: rec_cap
// records of 4 reals + j + key, then 7 ints per key).
// STENCIL: the batch of stencil sampling, decoded (drawn atoms, -1: none); BATCH:
// the list-drawn batch as the forward wrote it (batch_j), in place of the ranks
// and the shell rows.
template <typename real, bool FULL, bool WANT_LJ, bool BK, bool STENCIL, bool SKIN, bool BATCH>
__global__ __launch_bounds__(kCoopBlock) void k_pair_adjoint(
    int64_t n, int apw, PairParams<real> pp, const uint4* __restrict__ spos, const real* __restrict__ sqr,
    const uint4* __restrict__ spq, const int2* __restrict__ sxr, const int32_t* __restrict__ sxidx, const int32_t* __restrict__ core,
    const int32_t* __restrict__ ncore, int cap_core, const int32_t* __restrict__ shell,
    const int32_t* __restrict__ nshell, int cap_shell, const real* __restrict__ ljraw_g, int n_types, int p_shell,
    int p_stride, const uint16_t* __restrict__ ranks, const int32_t* __restrict__ batch_j, uint64_t t_core,
    uint64_t t_shell, real lj_cut, const real* __restrict__ gs, const double* __restrict__ gmean_d,
    real* __restrict__ gself, real* __restrict__ gscat, real* __restrict__ gqself, real* __restrict__ gqscat,
    double* __restrict__ ljpart, BucketArgs bk, int rec_cap)
{
    constexpr int NLJ = 2 * kMaxTypesGrad * kMaxTypesGrad;
    constexpr int NW = kCoopBlock / 64;
    __shared__ LJGrad<real> ljg[256];
    __shared__ int lj_row[16];  // 1 when some sigma of type t's row is nonzero (else no LJ term or gradient)
    __shared__ double ljacc[NW][NLJ];
    __shared__ int nrec;
    __shared__ double bmaxw[NW];
    extern __shared__ __align__(16) unsigned char bk_lds[];
    real* rc = (real*)bk_lds;                              // [rec_cap][4]
    int32_t* rj = (int32_t*)(rc + 4 * (size_t)rec_cap);    // [rec_cap] sorted index of j
    uint16_t* rk = (uint16_t*)(rj + rec_cap);              // [rec_cap] key
    const int span2 = bk.span * bk.span;
    const int nkeys = 2 * span2;
    int32_t* kcnt = (int32_t*)(rk + ((rec_cap + 1) & ~1));  // [nkeys] records per key
    int32_t* kcur = kcnt + nkeys;                           // [nkeys] write cursor
    int32_t* kbase = kcur + nkeys;                          // [nkeys] reserved offset in the bucket
    int32_t* kdst = kbase + nkeys;                          // [nkeys] destination row
    int32_t* kfirst = kdst + nkeys;                         // [nkeys] first atom of the row
    int32_t* kcap = kfirst + nkeys;                         // [nkeys] bucket capacity
    int32_t* kcount = kcap + nkeys;                         // [nkeys] atoms of the row in the LDS window
    const int nt2 = n_types * n_types;
    for (int t = threadIdx.x; t < nt2; t += kCoopBlock) ljg[t] = lj_grad_entry(ljraw_g[t], ljraw_g[nt2 + t], lj_cut);
    if (threadIdx.x < n_types) {
        int any = 0;
        for (int u = 0; u < n_types; ++u) any |= ljraw_g[threadIdx.x * n_types + u] != (real)0;
        lj_row[threadIdx.x] = any;
    }
    // the wavefront's index as a wave-uniform value (scalar atom indices and row addresses)
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (WANT_LJ)
        for (int t = lane; t < NLJ; t += 64) ljacc[wave][t] = 0.0;
    if (BK) {
        for (int t = threadIdx.x; t < nkeys; t += kCoopBlock) kcnt[t] = 0;
        if (threadIdx.x == 0) nrec = 0;
    }
    __syncthreads();
    const real mx = FULL ? (real)0 : (real)gmean_d[0];
    const real my = FULL ? (real)0 : (real)gmean_d[1];
    const real mz = FULL ? (real)0 : (real)gmean_d[2];
    const real ke = pp.ke;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t gw = blk * NW + wave;
    const int64_t a0 = gw * apw;
    const int64_t a1 = min(n, a0 + apw);
    // cell row of the block's first atom: the block's atoms lie in rows row0, row0 + 1, ...
    int row0 = 0;
    if (BK) {
        const int64_t f = min(blk * NW * apw, n - 1);
        int z, y;
        key_cell(bk, f, spos[f], z, y);
        row0 = z * bk.n_c + y;
    }
    real lane_max = 0;  // largest |component| of the records this lane staged
    const Atoms<real> at{spos, sqr, spq};
    // per-atom headers of the wavefront's atoms, one atom per lane, read once
    const int64_t ah = min(a0 + min(lane, apw - 1), n - 1);
    uint4 h_s;
    real h_q;
    at.get(ah, h_s, h_q);
    const real h_gx = gs[3 * ah], h_gy = gs[3 * ah + 1], h_gz = gs[3 * ah + 2];
    const int h_nsym = FULL ? nshell[ah] : ncore[ah];
    const int h_ns = FULL ? 0 : nshell[ah];
    const int2 h_x = sxr[ah];
    // shell weight N_S / p~ (1 when every member is taken), one division per lane
    const real h_w = h_ns > p_shell ? (real)((double)h_ns / (double)p_shell) : (real)1;
    // first-level indices of one atom's first pass: the lane's first symmetric-list
    // entry, its two batch ranks (or shell positions) and its first excluded partner
    auto first_level = [&](int64_t a, int t, int& jc, int& r0, int& r1, int& jx) {
        const int nsym = bcast(h_nsym, t);
        const int ns = bcast(h_ns, t);
        const int2 xr = make_int2(bcast(h_x.x, t), bcast(h_x.y, t));
        const bool sample = ns > p_shell;
        const int cnt = sample ? p_shell : ns;
        const uint16_t* rrow = ranks + a * (int64_t)p_stride;
        const int32_t* srow_sym = FULL ? shell + a * (int64_t)cap_shell : core + a * (int64_t)cap_core;
        // the excluded partners follow the symmetric list (entries nsym .. nsym + nx - 1)
        jc = lane < nsym ? srow_sym[lane] : (lane < nsym + xr.y ? sxidx[xr.x + lane - nsym] : -1);
        if (STENCIL || BATCH) {
            // the decoded batch (atoms; with stencil sampling -1 for i itself and i's
            // molecule) in place of ranks
            const int32_t* brow = batch_j + a * (int64_t)p_stride;
            r0 = lane < cnt ? brow[lane] : -1;
            r1 = lane + 64 < cnt ? brow[lane + 64] : -1;
        } else {
            r0 = lane < cnt ? (sample ? (int)rrow[lane] : lane) : -1;
            r1 = lane + 64 < cnt ? (sample ? (int)rrow[lane + 64] : lane + 64) : -1;
        }
        jx = -1;
    };
    int n_jc = -1, n_r0 = -1, n_r1 = -1, n_jx = -1;
    if (a0 < a1) first_level(a0, 0, n_jc, n_r0, n_r1, n_jx);
    for (int64_t a = a0; a < a1; ++a) {
        const int t_a = (int)(a - a0);
        const int jc = n_jc, r0 = n_r0, r1 = n_r1, jx = n_jx;
        // the next atom's first-level loads go out before this atom's dependent ones
        if (a + 1 < a1) first_level(a + 1, t_a + 1, n_jc, n_r0, n_r1, n_jx);
        const uint4 si = make_uint4(bcast(h_s.x, t_a), bcast(h_s.y, t_a), bcast(h_s.z, t_a),
                                    bcast(h_s.w, t_a));
        const int ti = (int)si.w;
        const int li = __mul24(ti, n_types);  // the atom's row of the LJ table
        int zi = 0, yi = 0;  // the atom's cell for the bucket keys
        if (BK) key_cell(bk, a, si, zi, yi);
        // with every sigma of its row zero, the atom has no LJ term and no LJ gradient
        const bool lj_i = WANT_LJ && lj_row[ti];
        const real qi = bcast(h_q, t_a);
        const real gx = bcast(h_gx, t_a), gy = bcast(h_gy, t_a), gz = bcast(h_gz, t_a);
        const real pgx = gx - mx, pgy = gy - my, pgz = gz - mz;  // G'_i
        const int nsym = bcast(h_nsym, t_a);
        const int ns = bcast(h_ns, t_a);
        const int2 xr = make_int2(bcast(h_x.x, t_a), bcast(h_x.y, t_a));
        real rx = 0, ry = 0, rz = 0, rq = 0;
        real acc_sig[kMaxTypesGrad], acc_eps[kMaxTypesGrad];
#pragma unroll
        for (int t = 0; t < kMaxTypesGrad; ++t) acc_sig[t] = acc_eps[t] = 0;
        const int32_t* srow_sym = FULL ? shell + a * (int64_t)cap_shell : core + a * (int64_t)cap_core;
        const int32_t* srow = shell + a * (int64_t)cap_shell;
        const bool sample = ns > p_shell;
        const int cnt = sample ? p_shell : ns;
        const real w = bcast(h_w, t_a);
        const uint16_t* rrow = ranks + a * (int64_t)p_stride;

        // symmetric sets (core pairs, or the whole list in full-list mode, and the
        // excluded pairs, xp): gathered. G'_j - G'_i = G_j - G_i, so the same
        // difference serves both.
        auto sym_pair = [&](uint4 sj, real qj, real gjx, real gjy, real gjz, bool xp) {
            real dx, dy, dz;
            separation(si, sj, pp.quantum, dx, dy, dz);
            const real r2 = dx * dx + dy * dy + dz * dz;
            const LJGrad<real>& L = ljg[li + (int)sj.w];
            const PairGrad<real> g = pair_grad(r2, ke * qi * qj, L, pp, xp);
            const real ex_ = gjx - gx, ey_ = gjy - gy, ez_ = gjz - gz;
            const real gd = dx * ex_ + dy * ey_ + dz * ez_;
            rx += g.phi * ex_ + g.dphi_r * dx * gd;
            ry += g.phi * ey_ + g.dphi_r * dy * gd;
            rz += g.phi * ez_ + g.dphi_r * dz * gd;
            rq += ke * qj * g.a_coul * gd;
            if (lj_i) {
                const real gdi = dx * pgx + dy * pgy + dz * pgz;
                const int tj = (int)sj.w;
#pragma unroll
                for (int t = 0; t < kMaxTypesGrad; ++t)
                    if (t == tj) {
                        acc_sig[t] += -L.eps * g.dc_dsig * gdi;
                        acc_eps[t] += -g.c_lj * gdi;
                    }
            }
        };
        // sampled shell pairs, one-sided: gathered for i, scattered for j
        auto shell_pair = [&](int j, uint4 sj, real qj) {
            real dx, dy, dz;
            separation(si, sj, pp.quantum, dx, dy, dz);
            const real r2 = dx * dx + dy * dy + dz * dz;
            const LJGrad<real>& L = ljg[li + (int)sj.w];
            const PairGrad<real> g = pair_grad(r2, ke * qi * qj, L, pp);
            const real gdi = dx * pgx + dy * pgy + dz * pgz;
            const real jx_ = w * (g.phi * pgx + g.dphi_r * dx * gdi);
            const real jy_ = w * (g.phi * pgy + g.dphi_r * dy * gdi);
            const real jz_ = w * (g.phi * pgz + g.dphi_r * dz * gdi);
            rx -= jx_;
            ry -= jy_;
            rz -= jz_;
            rq += w * (-ke * qj * g.a_coul) * gdi;
            const real jq_ = w * (-ke * qi * g.a_coul) * gdi;
            bool staged = false;
            if (BK) {
                // key: (source row - row0, row offset of j), on the cells of the build
                // when positions may have moved since
                const int nc_ = bk.n_c;
                const int src = zi * nc_ + yi - row0;  // wave-uniform
                int zj, yj;
                key_cell(bk, j, sj, zj, yj);
                const int kz = stencil_offset(zj, zi, bk.lo, bk.span, nc_) - bk.lo;
                const int ky = stencil_offset(yj, yi, bk.lo, bk.span, nc_) - bk.lo;
                if (src >= 0 && src < 2 && kz >= 0 && kz < bk.span && ky >= 0 && ky < bk.span) {
                    const int key = src * span2 + kz * bk.span + ky;
                    const uint64_t m = __ballot(1);
                    const int leader = __ffsll((unsigned long long)m) - 1;
                    int base = 0;
                    if (lane == leader) base = atomicAdd(&nrec, __popcll(m));
                    base = __shfl(base, leader, 64);
                    const int slot = base + __popcll(m & ((1ull << lane) - 1ull));
                    if (slot < rec_cap) {
                        rc[4 * slot + 0] = jx_;
                        rc[4 * slot + 1] = jy_;
                        rc[4 * slot + 2] = jz_;
                        rc[4 * slot + 3] = jq_;
                        rj[slot] = j;
                        rk[slot] = (uint16_t)key;
                        atomicAdd(&kcnt[key], 1);
                        lane_max = fmax(lane_max, fmax(fmax(fabs(jx_), fabs(jy_)), fmax(fabs(jz_), fabs(jq_))));
                        staged = true;
                    }
                }
            }
            if (!staged) {
                scatter_atomic(gscat, gqscat, (int64_t)j, jx_, jy_, jz_, jq_);
                if (BK) atomicAdd(bk.n_atomic, 1ull);
            }
            if (lj_i) {
                const int tj = (int)sj.w;
#pragma unroll
                for (int t = 0; t < kMaxTypesGrad; ++t)
                    if (t == tj) {
                        acc_sig[t] += w * (-L.eps * g.dc_dsig * gdi);
                        acc_eps[t] += w * (-g.c_lj * gdi);
                    }
            }
        };
        // first pass, every load of the dependent levels issued together (unused
        // slots load atom 0)
        const int js0 = (STENCIL || BATCH) ? r0 : ((!FULL && r0 >= 0) ? srow[r0] : -1);
        const int js1 = (STENCIL || BATCH) ? r1 : ((!FULL && r1 >= 0) ? srow[r1] : -1);
        const int ic = max(jc, 0), i0 = max(js0, 0), i1 = max(js1, 0), ix = max(jx, 0);
        uint4 pjc, pj0, pj1;
        real qjc, qj0, qj1;
        at.get(ic, pjc, qjc);
        const real gcx = gs[3 * (int64_t)ic], gcy = gs[3 * (int64_t)ic + 1], gcz = gs[3 * (int64_t)ic + 2];
        at.get(i0, pj0, qj0);
        at.get(i1, pj1, qj1);
        (void)jx;
        (void)ix;
        // skin: a symmetric-list entry counts inside r_core (r_shell for the full
        // list), a list shell entry inside the annulus, at these positions
        const uint64_t t_sym = FULL ? t_shell : t_core;
        auto sym_ok = [&](uint4 sj) { return !SKIN || dist2_q(si, sj) <= t_sym; };
        constexpr bool shell_test = STENCIL || SKIN;
        if (jc >= 0 && (lane >= nsym || sym_ok(pjc))) sym_pair(pjc, qjc, gcx, gcy, gcz, lane >= nsym);
        if (js0 >= 0 && (!shell_test || in_annulus(si, pj0, t_core, t_shell))) shell_pair(js0, pj0, qj0);
        if (js1 >= 0 && (!shell_test || in_annulus(si, pj1, t_core, t_shell))) shell_pair(js1, pj1, qj1);
        // the rest (long lists and large batches)
        for (int c = lane + 64; c < nsym + xr.y; c += 64) {
            const int j = c < nsym ? srow_sym[c] : sxidx[xr.x + c - nsym];
            uint4 sj;
            real qj;
            at.get(j, sj, qj);
            if (c >= nsym || sym_ok(sj))
                sym_pair(sj, qj, gs[3 * (int64_t)j], gs[3 * (int64_t)j + 1], gs[3 * (int64_t)j + 2], c >= nsym);
        }
        if (!FULL)
            for (int c = lane + 128; c < cnt; c += 64) {
                if (STENCIL || BATCH) {
                    const int j = batch_j[a * (int64_t)p_stride + c];
                    if (j < 0) continue;
                    uint4 sj;
                    real qj;
                    at.get(j, sj, qj);
                    if (!shell_test || in_annulus(si, sj, t_core, t_shell)) shell_pair(j, sj, qj);
                } else {
                    const int j = srow[sample ? (int)rrow[c] : c];
                    uint4 sj;
                    real qj;
                    at.get(j, sj, qj);
                    if (!SKIN || in_annulus(si, sj, t_core, t_shell)) shell_pair(j, sj, qj);
                }
            }
        rx = wave_sum_r(rx);
        ry = wave_sum_r(ry);
        rz = wave_sum_r(rz);
        rq = wave_sum_r(rq);
        if (lane == 0) {
            gself[3 * a + 0] = rx;
            gself[3 * a + 1] = ry;
            gself[3 * a + 2] = rz;
            gqself[a] = rq;
        }
        if (lj_i && ti < kMaxTypesGrad) {
#pragma unroll
            for (int t = 0; t < kMaxTypesGrad; ++t) {
                const real s_sig = wave_sum_r(acc_sig[t]);
                const real s_eps = wave_sum_r(acc_eps[t]);
                if (lane == 0) {
                    ljacc[wave][ti * kMaxTypesGrad + t] += (double)s_sig;
                    ljacc[wave][kMaxTypesGrad * kMaxTypesGrad + ti * kMaxTypesGrad + t] += (double)s_eps;
                }
            }
        }
    }
    if (WANT_LJ) {
        __syncthreads();
        if (threadIdx.x < NLJ) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) t += ljacc[w][threadIdx.x];
            ljpart[blk * (int64_t)NLJ + threadIdx.x] = t;
        }
    }
    if (BK) {
        // reserve one range per key in its destination row's bucket, and raise the
        // row's bound on |record| to this block's largest staged component
        double wmax = (double)lane_max;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) wmax = fmax(wmax, __shfl_xor(wmax, off, 64));
        if (lane == 0) bmaxw[wave] = wmax;
        __syncthreads();
        double bmax = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) bmax = fmax(bmax, bmaxw[w]);
        for (int t = threadIdx.x; t < nkeys; t += kCoopBlock) {
            const int c = kcnt[t];
            kcur[t] = 0;
            if (c == 0) continue;
            const int src = row0 + t / span2;
            const int rem = t % span2;
            const int dz = rem / bk.span + bk.lo, dy = rem % bk.span + bk.lo;
            int z = src / bk.n_c + dz, y = src % bk.n_c + dy;
            z = z < 0 ? z + bk.n_c : (z >= bk.n_c ? z - bk.n_c : z);
            y = y < 0 ? y + bk.n_c : (y >= bk.n_c ? y - bk.n_c : y);
            const int dst = z * bk.n_c + y;
            const int64_t b0 = bucket_start(bk, dst);
            const int64_t cap = bucket_start(bk, dst + 1) - b0;
            kdst[t] = dst;
            kfirst[t] = bk.cell_start[(int64_t)dst * bk.n_c];
            kcount[t] = min(bk.cell_start[(int64_t)(dst + 1) * bk.n_c] - kfirst[t], kBucketRowLds);
            kcap[t] = (int32_t)min(cap, (int64_t)INT32_MAX);
            const unsigned long long old = atomicAdd(&bk.cursor[dst], (unsigned long long)c);
            kbase[t] = (int32_t)min(old, (unsigned long long)INT32_MAX);
            atomicMax(&bk.rowmax[dst], (unsigned long long)__double_as_longlong(bmax));
        }
        __syncthreads();
        const int nr = min(nrec, rec_cap);
        real* out_c = (real*)bk.rec_c;
        for (int s = threadIdx.x; s < nr; s += kCoopBlock) {
            const int key = rk[s];
            const int64_t pos = (int64_t)kbase[key] + atomicAdd(&kcur[key], 1);
            const int j = rj[s];
            const int jrel = j - kfirst[key];
            const int dst = kdst[key];
            if (pos < kcap[key]) {
                const int64_t at = bucket_start(bk, dst) + pos;
                if (jrel >= 0 && jrel < kcount[key]) {
                    out_c[4 * at + 0] = rc[4 * s + 0];
                    out_c[4 * at + 1] = rc[4 * s + 1];
                    out_c[4 * at + 2] = rc[4 * s + 2];
                    out_c[4 * at + 3] = rc[4 * s + 3];
                    bk.rec_j[at] = (uint16_t)jrel;
                    continue;
                }
                bk.rec_j[at] = (uint16_t)0xffffu;  // reserved slot left empty
            }
            scatter_atomic(gscat, gqscat, (int64_t)j, rc[4 * s + 0], rc[4 * s + 1], rc[4 * s + 2], rc[4 * s + 3]);
            atomicAdd(bk.n_atomic, 1ull);
        }
    }
}

template <typename real>
struct Rec4;
template <>
struct Rec4<float> {
    using type = float4;
};
template <>
struct Rec4<double> {
    using type = double4;
};

// Reduce one destination row's bucket: 64-bit fixed-point LDS sums over its
// records, then added to the row's scatter gradients (the atomics of the
// fallback paths already in place). One block per row. With m a bound on the
// row's largest |record component| and nr its record count, values are scaled
// by 2^sh with m nr 2^sh < 2^62, so no partial sum overflows.
template <typename real>
__global__ __launch_bounds__(512) void k_bucket_reduce(BucketArgs bk, real* __restrict__ gscat,
                                                       real* __restrict__ gqscat)
{
    __shared__ long long acc[4 * kBucketRowLds];  // component-major: acc[d * kBucketRowLds + j]
    const int row = (int)xcd_block(blockIdx.x, gridDim.x);
    const int first = bk.cell_start[(int64_t)row * bk.n_c];
    const int count = bk.cell_start[(int64_t)(row + 1) * bk.n_c] - first;
    const int nl = min(count, kBucketRowLds);
    const int64_t b0 = bucket_start(bk, row);
    const int64_t cap = bucket_start(bk, row + 1) - b0;
    const int64_t nr = (int64_t)min(bk.cursor[row], (unsigned long long)cap);
    const double mx = __longlong_as_double((long long)bk.rowmax[row]);
    if (nr == 0 || !(mx > 0.0)) return;  // block-uniform: no records or all zero
    int e;
    frexp(mx * (double)nr, &e);  // mx nr < 2^e
    const int sh = 62 - e;
    for (int t = threadIdx.x; t < nl; t += 512)
        for (int d = 0; d < 4; ++d) acc[d * kBucketRowLds + t] = 0;
    __syncthreads();
    using V4 = typename Rec4<real>::type;
    const V4* rcg = (const V4*)bk.rec_c + b0;
    const uint16_t* rjg = bk.rec_j + b0;
    // kU records per thread per pass, all loads issued before the LDS updates
    // (indices past the end are clamped to the last record and then ignored)
    constexpr int kU = 4;
    for (int64_t s0 = 0; s0 < nr; s0 += 512 * kU) {
        int jr[kU];
        V4 v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t s = s0 + u * 512 + threadIdx.x;
            const int64_t sc = min(s, nr - 1);
            jr[u] = rjg[sc];
            v[u] = rcg[sc];
            if (s >= nr) jr[u] = nl;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (jr[u] >= nl) continue;
            atomicAdd((unsigned long long*)&acc[0 * kBucketRowLds + jr[u]],
                      (unsigned long long)__double2ll_rn(ldexp((double)v[u].x, sh)));
            atomicAdd((unsigned long long*)&acc[1 * kBucketRowLds + jr[u]],
                      (unsigned long long)__double2ll_rn(ldexp((double)v[u].y, sh)));
            atomicAdd((unsigned long long*)&acc[2 * kBucketRowLds + jr[u]],
                      (unsigned long long)__double2ll_rn(ldexp((double)v[u].z, sh)));
            atomicAdd((unsigned long long*)&acc[3 * kBucketRowLds + jr[u]],
                      (unsigned long long)__double2ll_rn(ldexp((double)v[u].w, sh)));
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nl; k += 512) {
        const int64_t j = first + k;
        gscat[3 * j + 0] += (real)ldexp((double)acc[0 * kBucketRowLds + k], -sh);
        gscat[3 * j + 1] += (real)ldexp((double)acc[1 * kBucketRowLds + k], -sh);
        gscat[3 * j + 2] += (real)ldexp((double)acc[2 * kBucketRowLds + k], -sh);
        gqscat[j] += (real)ldexp((double)acc[3 * kBucketRowLds + k], -sh);
    }
}

template <typename real, bool FULL, bool WANT_LJ, bool BK, bool STENCIL, bool BATCH = false>
static hipError_t launch_adj_t(irbe_ctx* h, uint64_t step, int apw, const BucketArgs& bk, int rec_cap, size_t lds)
{
    const int64_t n = h->cfg.n_atoms;
    PairParams<real> pp;
    pp.quantum = (real)h->geo.quantum;
    pp.beta = (real)h->cfg.ewald_beta;
    pp.cgauss = (real)(2.0 * h->cfg.ewald_beta / 1.7724538509055160273);
    pp.ke = (real)h->cfg.coulomb_k;
    hipError_t e = launch_draw(h, step);
    if (e != hipSuccess) return e;
    if (STENCIL && !h->batch_j_valid) {
        // the adjoint reads the batch decoded once (its blocks hold too few atoms
        // for the per-wavefront decode of the forward kernel to pay)
        e = launch_stencil_decode(h);
        if (e != hipSuccess) return e;
        h->batch_j_valid = true;
    }
    const int64_t waves = blocks_for(n, apw);
    const unsigned nb = (unsigned)blocks_for(waves, kCoopBlock / 64);
    if ((int64_t)nb > h->part_blocks) return hipErrorInvalidValue;
    h->adj_nb = nb;
#define IRBE_ADJ_ARGS                                                                                         \
    n, apw, pp, h->spos, (const real*)h->sq_r, h->spq, h->sxr, h->sxidx, h->core, h->ncore, h->cap_core, h->shell, \
        h->nshell, h->cap_shell, (const real*)h->lj_raw, h->cfg.n_types, h->cfg.p_shell, h->p_stride, h->ranks,  \
        h->batch_j, h->geo.t_core, h->geo.t_shell, (real)h->cfg.lj_cut, (const real*)h->gs, h->gmean,             \
        (real*)h->gself, (real*)h->gscat, (real*)h->gqself, (real*)h->gqscat, h->ljpart, bk, rec_cap
    if (h->geo.skin)
        k_pair_adjoint<real, FULL, WANT_LJ, BK, STENCIL, true, BATCH><<<nb, kCoopBlock, lds, h->stream>>>(IRBE_ADJ_ARGS);
    else
        k_pair_adjoint<real, FULL, WANT_LJ, BK, STENCIL, false, BATCH><<<nb, kCoopBlock, lds, h->stream>>>(IRBE_ADJ_ARGS);
    h->adj_used_batch = BATCH;
#undef IRBE_ADJ_ARGS
    e = hipGetLastError();
    if (e != hipSuccess || !BK) return e;
    const unsigned rows = (unsigned)((int64_t)bk.n_c * bk.n_c);
    k_bucket_reduce<real><<<rows, 512, 0, h->stream>>>(bk, (real*)h->gscat, (real*)h->gqscat);
    return hipGetLastError();
}

template <typename real, bool BK>
static hipError_t launch_adj_r(irbe_ctx* h, uint64_t step, bool want_lj, int apw, const BucketArgs& bk, int rec_cap,
                               size_t lds)
{
    if (h->full_list)
        return want_lj ? launch_adj_t<real, true, true, false, false>(h, step, apw, bk, 0, 0)
                       : launch_adj_t<real, true, false, false, false>(h, step, apw, bk, 0, 0);
    if (h->stencil) {
        // (the batch atoms the forward wrote when it was asked to, else decoded)
        const bool from_fwd = h->ranks_valid && h->ranks_step == step && h->batch_j_valid && h->batch_j_fwd;
        const hipError_t e = want_lj ? launch_adj_t<real, false, true, BK, true>(h, step, apw, bk, rec_cap, lds)
                                     : launch_adj_t<real, false, false, BK, true>(h, step, apw, bk, rec_cap, lds);
        h->adj_used_batch = from_fwd;
        return e;
    }
    // the batch atoms the forward wrote, when they are those of this step's ranks
    // (launch_draw keeps them unless it draws again); with 16-bit shell entries
    // the atoms at the ranks decoded once otherwise
    hipError_t e = launch_draw(h, step);
    if (e != hipSuccess) return e;
    const bool from_fwd = h->batch_j_valid && h->batch_j_fwd;
    if (h->shell16 && !h->batch_j_valid) {
        e = launch_list_decode(h);
        if (e != hipSuccess) return e;
        h->batch_j_valid = true;
        h->batch_j_fwd = false;
    }
    if (h->batch_j_valid) {
        e = want_lj ? launch_adj_t<real, false, true, BK, false, true>(h, step, apw, bk, rec_cap, lds)
                    : launch_adj_t<real, false, false, BK, false, true>(h, step, apw, bk, rec_cap, lds);
        h->adj_used_batch = from_fwd;
        return e;
    }
    return want_lj ? launch_adj_t<real, false, true, BK, false>(h, step, apw, bk, rec_cap, lds)
                   : launch_adj_t<real, false, false, BK, false>(h, step, apw, bk, rec_cap, lds);
}

hipError_t launch_pair_adjoint(irbe_ctx* h, uint64_t step, bool want_q, bool want_lj)
{
    (void)want_q;
    const int64_t n = h->cfg.n_atoms;
    hipError_t e = launch_fill_bytes0(h->stream, h->gscat, 3 * (size_t)n * h->real_size);
    if (e != hipSuccess) return e;
    e = launch_fill_bytes0(h->stream, h->gqscat, (size_t)n * h->real_size);
    if (e != hipSuccess) return e;
    // bucketed transpose of the shell scatter when a block of >= 8 atoms' records
    // fits the LDS staging area and the keys fit their table
    BucketArgs bk{};
    bk.n_c = h->geo.n_c;
    bk.lo = h->geo.lo;
    bk.span = h->geo.hi - h->geo.lo + 1;
    int p_eff = std::max(1, std::min(h->cfg.p_shell, std::max(h->shell_bound(), 1)));
    if (h->stencil) {
        // records only for the drawn atoms inside the shell: p~ times the shell's
        // share of the stencil volume, with a margin (the rest take the atomics)
        const double L = h->cfg.box_length, edge = L / h->geo.n_c;
        const double span = (double)(h->geo.hi - h->geo.lo + 1) * edge;
        const double rs = h->cfg.r_shell, rc = h->cfg.r_core;
        const double frac = std::min(1.0, 4.0 / 3.0 * 3.14159265358979323846 * (rs * rs * rs - rc * rc * rc) / (span * span * span));
        p_eff = std::max(1, std::min(p_eff, (int)std::ceil(1.3 * frac * h->cfg.p_shell)));
    }
    // records staged per block: room for the shell terms of every atom of the block
    // (kCoopBlock / 64 wavefronts of apw atoms, p_eff records each); apw fills a
    // budget that keeps five blocks on a CU, but is at least 2 (the bucketed
    // path's minimum) while the records fit the LDS limit (p~ <= 256 in FP32,
    // 128 in FP64; beyond, the shell terms take device atomics)
    const int waves_pb = kCoopBlock / 64;
    const int rec_budget = h->fp64 ? kBucketRecD : kBucketRecF;
    const int rec_max = h->fp64 ? kBucketRecMaxD : kBucketRecMaxF;
    int apw = std::min(kAtomsPerWave, std::max(2, rec_budget / (waves_pb * p_eff)));
    // a block's atoms within two cell rows, the source rows its keys cover: at most
    // 0.9 of a row's mean population per block (dilute small boxes), else the rest
    // of its shell records would take the atomic fallback
    const double row_atoms = (double)n / ((double)bk.n_c * (double)bk.n_c);
    apw = std::min(apw, std::max(2, (int)(0.9 * row_atoms / waves_pb)));
    if (waves_pb * apw * p_eff > rec_max) apw = rec_max / (waves_pb * p_eff);
    const int rec_cap = waves_pb * std::max(apw, 1) * p_eff;
    const int nkeys = 2 * bk.span * bk.span;
    const bool use_bk = !h->full_list && apw >= 2 && nkeys <= kBucketMaxKeys;
    size_t lds = 0;
    if (use_bk) {
        bk.p9 = 9 * (int64_t)p_eff;
        const int64_t rows = (int64_t)bk.n_c * bk.n_c;
        const int64_t total = ((int64_t)n * bk.p9 >> 3) + (int64_t)kBucketSlack * (rows + 1);
        e = ensure_buckets(h, total);
        if (e != hipSuccess) return e;
        e = launch_fill_i32(h->stream, (int32_t*)h->bk_cursor, 0, 4 * rows);
        if (e != hipSuccess) return e;
        e = launch_fill_i32(h->stream, (int32_t*)h->adj_atomics, 0, 2);
        if (e != hipSuccess) return e;
        bk.n_atomic = h->adj_atomics;
        bk.brow = h->geo.skin ? h->brow : nullptr;
        bk.cell_start = h->cell_start;
        bk.cursor = h->bk_cursor;
        bk.rowmax = h->bk_cursor + rows;
        bk.rec_c = h->bk_c;
        bk.rec_j = h->bk_j;
        lds = (size_t)rec_cap * (4 * h->real_size + 4) + (size_t)((rec_cap + 1) & ~1) * 2 + (size_t)nkeys * 7 * 4;
    }
    h->adj_all_atomic = !use_bk;
    if (h->fp64)
        return use_bk ? launch_adj_r<double, true>(h, step, want_lj, apw, bk, rec_cap, lds)
                      : launch_adj_r<double, false>(h, step, want_lj, kAtomsPerWave, bk, 0, 0);
    return use_bk ? launch_adj_r<float, true>(h, step, want_lj, apw, bk, rec_cap, lds)
                  : launch_adj_r<float, false>(h, step, want_lj, kAtomsPerWave, bk, 0, 0);
}

}  // namespace irbe
