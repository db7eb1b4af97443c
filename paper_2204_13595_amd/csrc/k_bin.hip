// Binning (Sec. 2.3: cells of edge >= r_core): fixed-point quantization of the
// positions, cell histogram, exclusive scan, scatter, in-cell ordering by
// (x coordinate, atom id), and the gather of a cell-sorted structure-of-arrays
// copy of the system.
#include <type_traits>

#include "irbe_device.hpp"
#include "irbe_internal.hpp"

namespace irbe {

int64_t blocks_for(int64_t n, int block) { return (n + block - 1) / block; }

__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u32x4(uint4* __restrict__ p, int64_t n4)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_fill_u8(uint8_t* __restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int32_t v, int64_t n)
{
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<(unsigned)blocks_for(n, kBlock), kBlock, 0, s>>>(p, v, n);
    return hipGetLastError();
}

// Zero a device buffer with kernels (no memset nodes, so the calls stay safe
// inside captured graphs).
hipError_t launch_fill_bytes0(hipStream_t s, void* p, size_t bytes)
{
    if (bytes == 0) return hipSuccess;
    const int64_t n4 = (int64_t)(bytes / 16);
    if (n4 > 0 && ((uintptr_t)p % 16) == 0) {
        k_fill_u32x4<<<(unsigned)blocks_for(n4, kBlock), kBlock, 0, s>>>((uint4*)p, n4);
        const size_t rest = bytes - (size_t)n4 * 16;
        if (rest) k_fill_u8<<<1, kBlock, 0, s>>>((uint8_t*)p + n4 * 16, (int64_t)rest);
    } else {
        k_fill_u8<<<(unsigned)blocks_for((int64_t)bytes, kBlock), kBlock, 0, s>>>((uint8_t*)p, (int64_t)bytes);
    }
    return hipGetLastError();
}

// s = rint(frac(x / L) * 2^32) mod 2^32, computed as rint((u - floor(u)) * 2^32)
// with u = x * (1/L). Contraction is off so the FP64 rounding is exactly that
// of the separate multiply and subtract.
__device__ __forceinline__ uint32_t quantize1(double x, double inv_l, bool& bad)
{
#pragma clang fp contract(off)
    if (!isfinite(x)) {
        bad = true;
        return 0u;
    }
    const double u = x * inv_l;
    const double f = u - floor(u);
    const double t = rint(f * 4294967296.0);
    return (uint32_t)((uint64_t)t & 0xffffffffull);
}

__device__ __forceinline__ uint32_t cell_coord(uint32_t s, int n_c) { return (uint32_t)(((uint64_t)s * (uint32_t)n_c) >> 32); }

template <typename real>
__global__ __launch_bounds__(kBlock) void k_quantize_hist(int64_t n, const real* __restrict__ pos, double inv_l,
                                                          int n_c, uint4* __restrict__ sq,
                                                          int32_t* __restrict__ cell_count,
                                                          int32_t* __restrict__ slot, uint32_t* err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool bad = false;
    const uint32_t sx = quantize1((double)pos[3 * i + 0], inv_l, bad);
    const uint32_t sy = quantize1((double)pos[3 * i + 1], inv_l, bad);
    const uint32_t sz = quantize1((double)pos[3 * i + 2], inv_l, bad);
    const uint32_t cell = (cell_coord(sz, n_c) * (uint32_t)n_c + cell_coord(sy, n_c)) * (uint32_t)n_c + cell_coord(sx, n_c);
    sq[i] = make_uint4(sx, sy, sz, cell);
    // the atom's place among its cell's atoms (any order: each cell is sorted later).
    // Consecutive lanes in one cell (a molecule's atoms, neighbouring molecules of an
    // ordered input) form a run whose first lane takes the run's places with one
    // atomic; the active lanes of a wavefront are a prefix of it.
    const int lane = (int)(threadIdx.x & 63u);
    const uint32_t prev = (uint32_t)__shfl_up((int)cell, 1, 64);
    const bool head = lane == 0 || prev != cell;
    const uint64_t heads = __builtin_amdgcn_ballot_w64(head);
    const uint64_t active = __builtin_amdgcn_ballot_w64(true);
    const uint64_t upto = (2ull << lane) - 1ull;  // lanes 0 .. lane (all ones for lane 63)
    const int first = 63 - __builtin_clzll(heads & upto);
    int base = 0;
    if (head) {
        const uint64_t later = heads & ~upto;
        const int end = later ? __builtin_ctzll(later) : 64 - __builtin_clzll(active);
        base = atomicAdd(&cell_count[cell], end - lane);
    }
    slot[i] = __shfl(base, first, 64) + (lane - first);
    if (bad) atomicOr(err, ERR_NONFINITE);
}

// Exclusive scan, 1024 elements per block; the block total goes to sums[b].
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(kScanBlock) void k_scan_block(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                           int32_t* __restrict__ sums, int64_t n)
{
    __shared__ int32_t wave_tot[kScanBlock / 64];
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t v = i < n ? in[i] : 0;
    int32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wave_tot[wave] = x;
    __syncthreads();
    if (wave == 0) {
        int32_t t = lane < kScanBlock / 64 ? wave_tot[lane] : 0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(t, off, 64);
            if (lane >= off) t += y;
        }
        if (lane < kScanBlock / 64) wave_tot[lane] = t;
    }
    __syncthreads();
    const int32_t base = wave > 0 ? wave_tot[wave - 1] : 0;
    if (i < n) out[i] = base + x - v;
    if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = base + x;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_add(int32_t* __restrict__ out, const int32_t* __restrict__ sums, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    if (i < n && blockIdx.x > 0) out[i] += sums[blockIdx.x];
}

// Exclusive scan of in[0..n) into out[0..n]; out[n] = total. levels holds the
// per-level block-sum buffers sized at handle creation.
static hipError_t scan_exclusive(irbe_ctx* h, const int32_t* in, int32_t* out, int64_t n)
{
    const int64_t nb = blocks_for(n, kScanBlock);
    int32_t* sums = h->scan_levels[0];
    k_scan_block<<<(unsigned)nb, kScanBlock, 0, h->stream>>>(in, out, sums, n);
    // scan the block totals level by level
    std::vector<int64_t> lens{nb};
    int level = 0;
    while (lens.back() > 1) {
        const int64_t m = lens.back();
        const int64_t mb = blocks_for(m, kScanBlock);
        int32_t* cur = h->scan_levels[level];
        int32_t* nxt = h->scan_levels[level + 1];
        k_scan_block<<<(unsigned)mb, kScanBlock, 0, h->stream>>>(cur, cur, nxt, m);
        lens.push_back(mb);
        ++level;
    }
    for (int lv = level - 1; lv >= 0; --lv) {
        const int64_t m = lens[lv];
        k_scan_add<<<(unsigned)blocks_for(m, kScanBlock), kScanBlock, 0, h->stream>>>(h->scan_levels[lv],
                                                                                      h->scan_levels[lv + 1], m);
    }
    k_scan_add<<<(unsigned)nb, kScanBlock, 0, h->stream>>>(out, h->scan_levels[0], n);
    // total: out[n] = out[n-1] + in[n-1]
    return hipGetLastError();
}

__global__ void k_scan_total(const int32_t* __restrict__ in, int32_t* __restrict__ out, int64_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

__global__ __launch_bounds__(kBlock) void k_scatter(int64_t n, const uint4* __restrict__ sq,
                                                    const int32_t* __restrict__ cell_start,
                                                    const int32_t* __restrict__ slot, int32_t* __restrict__ perm)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    perm[cell_start[sq[i].w] + slot[i]] = (int32_t)i;
}

// Order each cell's atoms by (fixed-point x coordinate, atom id); sorting by x
// lets the list build trim each atom's candidate range to its exact x extent.
// Slot k of the cell-grouped order `in` holds atom i; its place in the cell is
// the number of the cell's atoms with a smaller key (keys are distinct, as the
// ids are): one thread per atom over the cell's few tens of atoms, whose loads
// the threads of one cell share.
__global__ __launch_bounds__(kBlock) void k_cell_rank(int64_t n, const int32_t* __restrict__ cell_start,
                                                      const uint4* __restrict__ sq, const int32_t* __restrict__ in,
                                                      int32_t* __restrict__ perm)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t i = in[k];
    const uint4 si = sq[i];
    const int32_t b = cell_start[si.w], e = cell_start[si.w + 1];
    int32_t r = 0;
    for (int32_t t = b; t < e; ++t) {
        const int32_t u = in[t];
        const uint32_t xu = sq[u].x;
        r += (xu < si.x || (xu == si.x && u < i)) ? 1 : 0;
    }
    perm[b + r] = i;
}

// The FP32 pair kernels' record of an atom: the fixed-point coordinates and the
// charge rounded to 19 mantissa bits (to nearest, ties away from zero), whose
// freed 4 low bits carry the type (n_types <= 16).
__device__ __forceinline__ uint4 pos_charge_record(uint4 s, float q, int32_t type)
{
    const uint32_t b = (__float_as_uint(q) + 8u) & ~15u;
    return make_uint4(s.x, s.y, s.z, b | ((uint32_t)type & 15u));
}

template <typename real>
__global__ __launch_bounds__(kBlock) void k_gather_sorted(int64_t n, const int32_t* __restrict__ perm,
                                                          const uint4* __restrict__ sq,
                                                          const int32_t* __restrict__ type,
                                                          const real* __restrict__ q, const int32_t* __restrict__ mol,
                                                          const int32_t* __restrict__ xoff,
                                                          uint4* __restrict__ spos, real* __restrict__ sqr,
                                                          uint4* __restrict__ spq, int32_t* __restrict__ smol,
                                                          int2* __restrict__ sxr, int32_t* __restrict__ rank,
                                                          int n_c, int32_t* __restrict__ brow)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t i = perm[k];
    const uint4 s = sq[i];
    if (brow) {
        // the cell's (z, y) at this build (s.w is the cell id)
        const uint32_t row = s.w / (uint32_t)n_c;
        brow[k] = (int32_t)(((row / (uint32_t)n_c) << 16) | (row % (uint32_t)n_c));
    }
    spos[k] = make_uint4(s.x, s.y, s.z, (uint32_t)type[i]);
    sqr[k] = q[i];
    if (std::is_same<real, float>::value) spq[k] = pos_charge_record(s, (float)q[i], type[i]);
    smol[k] = mol[i];
    sxr[k] = make_int2(xoff[i], xoff[i + 1] - xoff[i]);
    rank[i] = (int32_t)k;
}

// Excluded partners as sorted indices (same layout as the caller-order table).
__global__ __launch_bounds__(kBlock) void k_excl_sorted(int64_t n_excl, const int32_t* __restrict__ xidx,
                                                        const int32_t* __restrict__ rank, int32_t* __restrict__ sxidx)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n_excl) sxidx[e] = rank[xidx[e]];
}

hipError_t launch_bin(irbe_ctx* h, const void* pos)
{
    const int64_t n = h->cfg.n_atoms;
    const unsigned nb = (unsigned)blocks_for(n, kBlock);
    hipError_t e = launch_fill_i32(h->stream, h->cell_count, 0, h->geo.n_cells);
    if (e != hipSuccess) return e;
    if (h->fp64)
        k_quantize_hist<double><<<nb, kBlock, 0, h->stream>>>(n, (const double*)pos, h->geo.inv_l, h->geo.n_c, h->sq,
                                                              h->cell_count, h->smol, h->err);
    else
        k_quantize_hist<float><<<nb, kBlock, 0, h->stream>>>(n, (const float*)pos, h->geo.inv_l, h->geo.n_c, h->sq,
                                                             h->cell_count, h->smol, h->err);
    e = scan_exclusive(h, h->cell_count, h->cell_start, h->geo.n_cells);
    if (e != hipSuccess) return e;
    k_scan_total<<<1, 64, 0, h->stream>>>(h->cell_count, h->cell_start, h->geo.n_cells);
    // the atoms grouped by cell into rank, each at the place its histogram atomic
    // returned (held in smol), then each cell ordered into perm; rank and smol are
    // free until k_gather_sorted rewrites them
    k_scatter<<<nb, kBlock, 0, h->stream>>>(n, h->sq, h->cell_start, h->smol, h->rank);
    k_cell_rank<<<nb, kBlock, 0, h->stream>>>(n, h->cell_start, h->sq, h->rank, h->perm);
    if (h->fp64)
        k_gather_sorted<double><<<nb, kBlock, 0, h->stream>>>(n, h->perm, h->sq, h->type_orig, (const double*)h->q_orig,
                                                              h->mol_orig, h->xoff, h->spos, (double*)h->sq_r,
                                                              nullptr, h->smol, h->sxr, h->rank, h->geo.n_c,
                                                              h->brow);
    else
        k_gather_sorted<float><<<nb, kBlock, 0, h->stream>>>(n, h->perm, h->sq, h->type_orig, (const float*)h->q_orig,
                                                             h->mol_orig, h->xoff, h->spos, (float*)h->sq_r, h->spq,
                                                             h->smol, h->sxr, h->rank, h->geo.n_c, h->brow);
    if (h->n_excl > 0)
        k_excl_sorted<<<(unsigned)blocks_for(h->n_excl, kBlock), kBlock, 0, h->stream>>>(h->n_excl, h->xidx, h->rank,
                                                                                        h->sxidx);
    return hipGetLastError();
}

// Re-quantize positions for a force evaluation on the lists of the last build:
// the sorted order (perm) is kept, positions and charges are refreshed.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_requantize(int64_t n, const real* __restrict__ pos, double inv_l,
                                                       const int32_t* __restrict__ rank,
                                                       const int32_t* __restrict__ type, const real* __restrict__ q,
                                                       uint4* __restrict__ sq, uint4* __restrict__ spos,
                                                       real* __restrict__ sqr, uint4* __restrict__ spq, uint32_t* err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool bad = false;
    const uint32_t sx = quantize1((double)pos[3 * i + 0], inv_l, bad);
    const uint32_t sy = quantize1((double)pos[3 * i + 1], inv_l, bad);
    const uint32_t sz = quantize1((double)pos[3 * i + 2], inv_l, bad);
    const int32_t k = rank[i];
    sq[i] = make_uint4(sx, sy, sz, sq[i].w);
    spos[k] = make_uint4(sx, sy, sz, (uint32_t)type[i]);
    sqr[k] = q[i];
    if (std::is_same<real, float>::value)
        spq[k] = pos_charge_record(make_uint4(sx, sy, sz, 0u), (float)q[i], type[i]);
    if (bad) atomicOr(err, ERR_NONFINITE);
}

hipError_t launch_requantize(irbe_ctx* h, const void* pos)
{
    const int64_t n = h->cfg.n_atoms;
    const unsigned nb = (unsigned)blocks_for(n, kBlock);
    if (h->fp64)
        k_requantize<double><<<nb, kBlock, 0, h->stream>>>(n, (const double*)pos, h->geo.inv_l, h->rank, h->type_orig,
                                                           (const double*)h->q_orig, h->sq, h->spos,
                                                           (double*)h->sq_r, nullptr, h->err);
    else
        k_requantize<float><<<nb, kBlock, 0, h->stream>>>(n, (const float*)pos, h->geo.inv_l, h->rank, h->type_orig,
                                                          (const float*)h->q_orig, h->sq, h->spos, (float*)h->sq_r,
                                                          h->spq, h->err);
    return hipGetLastError();
}

// Sum of q^2 (FP64) for the self energy.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_sum_q2_part(int64_t n, const real* __restrict__ q, double* __restrict__ part)
{
    __shared__ double lds[kBlock / 64];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        const double x = (double)q[i];
        v = x * x;
    }
    double vals[1] = {v};
    double out;
    block_sum_vec<1, kBlock>(vals, lds, threadIdx.x, out);
    if (threadIdx.x == 0) part[blockIdx.x] = out;
}

__global__ __launch_bounds__(kReduceBlock) void k_sum_part(int64_t nb, const double* __restrict__ part, double* __restrict__ out)
{
    __shared__ double lds[kReduceBlock / 64];
    double v = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += kReduceBlock) v += part[b];
    double vals[1] = {v};
    double o;
    block_sum_vec<1, kReduceBlock>(vals, lds, threadIdx.x, o);
    if (threadIdx.x == 0) out[0] = o;
}

hipError_t launch_sum_q2(irbe_ctx* h)
{
    const int64_t n = h->cfg.n_atoms;
    const int64_t nb = blocks_for(n, kBlock);
    if (h->fp64)
        k_sum_q2_part<double><<<(unsigned)nb, kBlock, 0, h->stream>>>(n, (const double*)h->q_orig, h->q2part);
    else
        k_sum_q2_part<float><<<(unsigned)nb, kBlock, 0, h->stream>>>(n, (const float*)h->q_orig, h->q2part);
    k_sum_part<<<1, kReduceBlock, 0, h->stream>>>(nb, h->q2part, h->sumq2);
    return hipGetLastError();
}

}  // namespace irbe
