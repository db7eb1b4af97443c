// Core and shell lists (Sec. 2.3): C(i) = {j != i : r_ij <= r_core} and
// S(i) = {j : r_core < r_ij <= r_shell}, same-molecule pairs removed, in the
// canonical order "stencil cell offset (dz, dy, dx) lexicographic, then the
// atoms of each cell in cell order (by fixed-point x coordinate, then id)". One traversal of the shell stencil yields both
// lists: the 27 core cells are visited in their own lexicographic order
// inside it. Membership is exact: uint64 squared separations in quanta of
// L / 2^32 against integer thresholds (an FP32 estimate settles every
// candidate that is not within 2^-19 of a threshold; the rest are tested
// exactly).
//
// One wavefront handles the atoms of G consecutive cells of one cell row (one
// lane per atom). For every stencil row (dz, dy) the union of the lanes' x
// ranges is staged in LDS; each lane scans only the cells its own sphere can
// reach (per-atom pruning of rows and of the x range from exact cell-boundary
// distances; inside the first and last cell of the range, a binary search on
// the x-sorted cell trims the range to the atom's exact x extent), which
// leaves the member order unchanged.
//
// Layout: fixed-capacity rows (row k of atom k in cell order), entries are
// cell-sorted atom indices, written four at a time. Counts beyond the capacity
// are still counted, so the host can grow the rows and rebuild.
#include <algorithm>

#include "irbe_device.hpp"
#include "irbe_internal.hpp"

namespace irbe {

constexpr int kListWave = 64;
constexpr int kTileCap = 256;  // staged candidates per pass

__device__ __forceinline__ uint64_t dist2_exact(uint4 a, uint4 b)
{
    const int32_t dx = (int32_t)(b.x - a.x);
    const int32_t dy = (int32_t)(b.y - a.y);
    const int32_t dz = (int32_t)(b.z - a.z);
    return (uint64_t)((int64_t)dx * dx) + (uint64_t)((int64_t)dy * dy) + (uint64_t)((int64_t)dz * dz);
}

__device__ __forceinline__ int wrap(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// Append v to a row through a 4-entry register buffer (16-byte stores).
struct RowWriter {
    int32_t* row;
    int cap;
    int count;
    int b0, b1, b2;

    __device__ __forceinline__ void push(int v)
    {
        const int slot = count & 3;
        if (slot == 0) b0 = v;
        else if (slot == 1) b1 = v;
        else if (slot == 2) b2 = v;
        else if (count < cap) *(int4*)(row + (count - 3)) = make_int4(b0, b1, b2, v);
        ++count;
    }

    __device__ __forceinline__ void flush()
    {
        const int slot = count & 3;
        const int base = count - slot;
        if (slot > 0 && base < cap) row[base] = b0;
        if (slot > 1 && base + 1 < cap) row[base + 1] = b1;
        if (slot > 2 && base + 2 < cap) row[base + 2] = b2;
    }
};

// Distance (quanta) from coordinate s to the slab of cell c on one axis when
// the slab lies at offset d (d > 0 above, d < 0 below); bound[c] is the first
// coordinate of cell c (bound[n_c] wraps to 0).
__device__ __forceinline__ uint32_t slab_gap(uint32_t s, int d, int c, const uint32_t* bound)
{
    if (d > 0) return bound[c] - s;
    if (d < 0) return s - (bound[c + 1] - 1u);
    return 0u;
}

template <bool FULL>
__global__ __launch_bounds__(kListWave) void k_build_lists_tiled(
    int n_c, int lo, int hi, int G, int prune, uint64_t t_core, uint64_t t_shell, float tfc_lo, float tfc_hi,
    float tfs_lo, float tfs_hi,
    const uint4* __restrict__ spos, const int32_t* __restrict__ smol, const int32_t* __restrict__ cell_start,
    const uint32_t* __restrict__ bound_g, int cap_core, int cap_shell, int32_t* __restrict__ core,
    int32_t* __restrict__ ncore, int32_t* __restrict__ shell, int32_t* __restrict__ nshell,
    int32_t* __restrict__ maxcnt)
{
    __shared__ uint4 tile[kTileCap];
    __shared__ int32_t tmol[kTileCap];
    const uint32_t* bound = bound_g;  // indexed by wave-uniform cell coordinates
    const int lane = threadIdx.x;
    const int groups_per_row = (n_c + G - 1) / G;
    const int g = (int)xcd_block(blockIdx.x, gridDim.x);
    const int rowid = g / groups_per_row;
    const int cz = rowid / n_c, cy = rowid % n_c;
    const int x0 = (g % groups_per_row) * G;
    const int gr = min(G, n_c - x0);
    const int home = (cz * n_c + cy) * n_c;
    const int a0 = cell_start[home + x0], a1 = cell_start[home + x0 + gr];
    const int span_c = hi - lo + 1;           // cells per lane's x range
    const int span_u = gr - 1 + span_c;       // cells of the union x range
    const int xu0 = wrap(x0 + lo, n_c);       // first cell of the union
    const int lenA = min(span_u, n_c - xu0);  // cells before the wrap
    int maxc = 0, maxs = 0;
    for (int chunk = a0; chunk < a1; chunk += kListWave) {
        const int k = chunk + lane;
        const bool act = k < a1;
        const uint4 si = act ? spos[k] : make_uint4(0, 0, 0, 0);
        const int32_t mi = act ? smol[k] : -1;
        const int cx = (int)(((uint64_t)si.x * (uint32_t)n_c) >> 32);
        const int ti = act ? wrap(cx - x0, n_c) : 0;  // lane's home cell in [0, gr)
        int32_t* crow = core + (int64_t)(act ? k : 0) * cap_core;  // core entries are few: stored directly
        int nc = 0;
        RowWriter ws{shell + (int64_t)(act ? k : 0) * cap_shell, cap_shell, 0, 0, 0, 0};
        for (int dz = lo; dz <= hi; ++dz) {
            const int z = wrap(cz + dz, n_c);
            const float gz = prune ? (float)slab_gap(si.z, dz, z, bound) : 0.0f;
            for (int dy = lo; dy <= hi; ++dy) {
                const int y = wrap(cy + dy, n_c);
                const int row = (z * n_c + y) * n_c;
                // lane's candidate cells in this row: tile cells [u_lo, u_hi]
                int u_lo = ti, u_hi = ti + span_c - 1;
                bool need = act;
                int32_t ext_i = 0x7fffffff;  // x half-extent (quanta) of the lane's sphere in this row
                if (prune && act) {
                    const float gy = (float)slab_gap(si.y, dy, y, bound);
                    const float rem = tfs_hi - gy * gy - gz * gz;
                    if (rem < 0.0f) {
                        need = false;
                    } else {
                        const uint32_t ext = (uint32_t)(sqrtf(rem) * 1.000002f) + 2u;
                        ext_i = (int32_t)ext;
                        const int cl = (int)(((uint64_t)(uint32_t)(si.x - ext) * (uint32_t)n_c) >> 32);
                        const int ch = (int)(((uint64_t)(uint32_t)(si.x + ext) * (uint32_t)n_c) >> 32);
                        int ol = cl - cx, oh = ch - cx;
                        if (ol > n_c / 2) ol -= n_c;
                        if (ol < -n_c / 2) ol += n_c;
                        if (oh > n_c / 2) oh -= n_c;
                        if (oh < -n_c / 2) oh += n_c;
                        u_lo = ti + (max(ol, lo) - lo);
                        u_hi = ti + (min(oh, hi) - lo);
                    }
                }
                if (__ballot(need) == 0) continue;
                // union of the x ranges: segment A (cells xu0 .. xu0+lenA-1), then B (cells 0 ..)
                const int jA = cell_start[row + xu0];
                const int eA = cell_start[row + xu0 + lenA];
                const int lenB = span_u - lenA;
                const int jB = cell_start[row];
                const int eB = lenB > 0 ? cell_start[row + lenB] : jB;
                const int nA = eA - jA;
                const int total = nA + (eB - jB);
                // lane's range in tile positions; tpos(u) = position of the first atom of tile cell u
                auto tpos = [&](int u) {
                    return u < lenA ? cell_start[row + xu0 + u] - jA : nA + cell_start[row + u - lenA] - jB;
                };
                int p_lo = 0, p_hi = 0, pc1 = 0, pc2 = 0;
                if (need) {
                    p_lo = tpos(u_lo);
                    p_hi = tpos(u_hi + 1);
                    pc1 = u_lo < u_hi ? tpos(u_lo + 1) : p_hi;  // end of the first cell
                    pc2 = u_lo < u_hi ? tpos(u_hi) : p_lo;      // start of the last cell
                }
                for (int base = 0; base < total; base += kTileCap) {
                    const int cnt = min(kTileCap, total - base);
                    __syncthreads();
                    for (int t = lane; t < cnt; t += kListWave) {
                        const int p = base + t;
                        const int j = p < nA ? jA + p : jB + (p - nA);
                        tile[t] = spos[j];
                        tmol[t] = smol[j];
                    }
                    __syncthreads();
                    if (prune && need && total <= kTileCap) {
                        // the cells are x-sorted: trim the first and the last cell of the range
                        int a = p_lo, b = pc1;
                        while (a < b) {
                            const int m = (a + b) >> 1;
                            if ((int32_t)(tile[m].x - si.x) < -ext_i) a = m + 1;
                            else b = m;
                        }
                        p_lo = a;
                        a = max(pc2, p_lo);
                        b = p_hi;
                        while (a < b) {
                            const int m = (a + b) >> 1;
                            if ((int32_t)(tile[m].x - si.x) <= ext_i) a = m + 1;
                            else b = m;
                        }
                        p_hi = a;
                    }
                    const int s0 = max(p_lo, base), s1 = min(p_hi, base + cnt);
                    // classify one staged candidate (FP32 estimate, exact test near a threshold)
                    auto visit = [&](int p, uint4 sj) {
                        const float fx = (float)(int32_t)(sj.x - si.x);
                        const float fy = (float)(int32_t)(sj.y - si.y);
                        const float fz = (float)(int32_t)(sj.z - si.z);
                        const float d2f = fx * fx + fy * fy + fz * fz;
                        if (d2f > tfs_hi) return;
                        const int j = p < nA ? jA + p : jB + (p - nA);
                        if (j == k || (mi >= 0 && tmol[p - base] == mi)) return;
                        int cls;
                        if (FULL) {
                            cls = d2f < tfs_lo ? 2 : (dist2_exact(si, sj) <= t_shell ? 2 : 0);
                        } else if (d2f < tfc_lo) {
                            cls = 1;
                        } else if (d2f > tfc_hi && d2f < tfs_lo) {
                            cls = 2;
                        } else {
                            const uint64_t d2 = dist2_exact(si, sj);
                            cls = d2 <= t_core ? 1 : (d2 <= t_shell ? 2 : 0);
                        }
                        if (cls == 1) {
                            if (nc < cap_core) crow[nc] = j;
                            ++nc;
                        } else if (cls == 2) {
                            ws.push(j);
                        }
                    };
                    int p = s0;
                    for (; p + 4 <= s1; p += 4) {
                        const uint4 q0 = tile[p - base], q1 = tile[p + 1 - base];
                        const uint4 q2 = tile[p + 2 - base], q3 = tile[p + 3 - base];
                        visit(p, q0);
                        visit(p + 1, q1);
                        visit(p + 2, q2);
                        visit(p + 3, q3);
                    }
                    for (; p < s1; ++p) visit(p, tile[p - base]);
                }
            }
        }
        if (act) {
            ws.flush();
            ncore[k] = nc;
            nshell[k] = ws.count;
            maxc = max(maxc, nc);
            maxs = max(maxs, ws.count);
        }
    }
    // one atomic per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        maxc = max(maxc, __shfl_xor(maxc, off, 64));
        maxs = max(maxs, __shfl_xor(maxs, off, 64));
    }
    if (lane == 0) {
        atomicMax(&maxcnt[0], maxc);
        atomicMax(&maxcnt[1], maxs);
    }
}

hipError_t launch_build_lists(irbe_ctx* h)
{
    const Geometry& g = h->geo;
    const int n_c = g.n_c;
    const bool narrow = 2 * g.reach + 1 <= n_c;
    const int G = narrow ? std::min(4, n_c - 2 * g.reach) : 1;
    const int prune = narrow ? 1 : 0;
    const int64_t groups = (int64_t)n_c * n_c * ((n_c + G - 1) / G);
    // FP32 thresholds with a relative margin of 2e-6, far above the FP32
    // rounding of the squared separations (< 3e-7): outside the bands the FP32
    // decision equals the exact one, inside them the exact test decides.
    const float tfc = (float)g.t_core, tfs = (float)g.t_shell;
    const float tfc_lo = tfc * 0.999998f, tfc_hi = tfc * 1.000002f;
    const float tfs_lo = tfs * 0.999998f, tfs_hi = tfs * 1.000002f;
    if (h->full_list)
        k_build_lists_tiled<true><<<(unsigned)groups, kListWave, 0, h->stream>>>(
            n_c, g.lo, g.hi, G, prune, g.t_core, g.t_shell, tfc_lo, tfc_hi, tfs_lo, tfs_hi, h->spos, h->smol, h->cell_start, h->cell_bound,
            h->cap_core, h->cap_shell, h->core, h->ncore, h->shell, h->nshell, h->maxcnt);
    else
        k_build_lists_tiled<false><<<(unsigned)groups, kListWave, 0, h->stream>>>(
            n_c, g.lo, g.hi, G, prune, g.t_core, g.t_shell, tfc_lo, tfc_hi, tfs_lo, tfs_hi, h->spos, h->smol, h->cell_start, h->cell_bound,
            h->cap_core, h->cap_shell, h->core, h->ncore, h->shell, h->nshell, h->maxcnt);
    return hipGetLastError();
}

}  // namespace irbe
