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

// Distance (quanta) from coordinate s to the slab of cell c on one axis when
// the slab lies at offset d (d > 0 above, d < 0 below); bound[c] is the first
// coordinate of cell c (bound[n_c] wraps to 0).
__device__ __forceinline__ uint32_t slab_gap(uint32_t s, int d, int c, const uint32_t* bound)
{
    if (d > 0) return bound[c] - s;
    if (d < 0) return s - (bound[c + 1] - 1u);
    return 0u;
}

// Number of set bits of mask below this lane.
__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
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
    __shared__ uint4 tile[kTileCap];      // staged candidates: fixed-point x, y, z and sorted index
    __shared__ int32_t tmol[kTileCap];    // candidate's exclusion id (molecule, or -2 - index)
    __shared__ uint4 apos[kListWave];     // atom's x, y, z and exclusion id
    __shared__ int2 arng[kListWave];      // atom's candidate range in the tile
    __shared__ int2 acnt[kListWave];      // atom's core / shell list lengths so far
    const uint32_t* bound = bound_g;  // indexed by wave-uniform cell coordinates
    const int lane = threadIdx.x;
    const int half = lane >> 5, hl = lane & 31;
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
        const int na = min(kListWave, a1 - chunk);
        const uint4 si = act ? spos[k] : make_uint4(0, 0, 0, 0);
        const int32_t mi = act ? smol[k] : -1;
        const int cx = (int)(((uint64_t)si.x * (uint32_t)n_c) >> 32);
        const int ti = act ? wrap(cx - x0, n_c) : 0;  // lane's home cell in [0, gr)
        apos[lane] = make_uint4(si.x, si.y, si.z, (uint32_t)(mi >= 0 ? mi : -2 - k));
        acnt[lane] = make_int2(0, 0);
        for (int dz = lo; dz <= hi; ++dz) {
            const int z = wrap(cz + dz, n_c);
            const float gz = prune ? (float)slab_gap(si.z, dz, z, bound) : 0.0f;
            for (int dy = lo; dy <= hi; ++dy) {
                const int y = wrap(cy + dy, n_c);
                const int row = (z * n_c + y) * n_c;
                const bool core_row = !FULL && dz >= -1 && dz <= 1 && dy >= -1 && dy <= 1;
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
                        const uint4 sj = spos[j];
                        const int32_t mj = smol[j];
                        tile[t] = make_uint4(sj.x, sj.y, sj.z, (uint32_t)j);
                        tmol[t] = mj >= 0 ? mj : -2 - j;
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
                    // this tile's part of the lane's range, in tile coordinates
                    const int s0 = need ? max(p_lo, base) - base : 0;
                    const int s1 = need ? min(p_hi, base + cnt) - base : 0;
                    arng[lane] = make_int2(s0, max(s1, s0));
                    __syncthreads();
                    // two atoms at a time, one per half-wave; the lanes of a half run over
                    // the atom's candidates and the members are compacted in candidate order
                    for (int pa = 0; pa < na; pa += 2) {
                        const int ka = min(pa + half, na - 1);
                        const bool hv = pa + half < na;
                        const int2 rg = arng[ka];
                        const int len = hv ? rg.y - rg.x : 0;
                        const int maxlen = max(len, __shfl_xor(len, 32, 64));
                        if (maxlen == 0) continue;
                        const uint4 sa = apos[ka];
                        const int32_t ma = (int32_t)sa.w;
                        const int kk = chunk + ka;
                        int2 c = acnt[ka];
                        int32_t* srow = shell + (int64_t)kk * cap_shell;
                        int32_t* crow = core + (int64_t)kk * cap_core;
                        for (int c0 = 0; c0 < maxlen; c0 += 32) {
                            const int q = (rg.x + c0 + hl) & (kTileCap - 1);
                            const uint4 sj = tile[q];
                            const int32_t mj = tmol[q];
                            const int32_t ddx = (int32_t)(sj.x - sa.x);
                            const int32_t ddy = (int32_t)(sj.y - sa.y);
                            const int32_t ddz = (int32_t)(sj.z - sa.z);
                            const float fx = (float)ddx, fy = (float)ddy, fz = (float)ddz;
                            const float d2f = fx * fx + fy * fy + fz * fz;
                            const bool keep = c0 + hl < len && mj != ma;
                            bool in_core = !FULL && keep && d2f < tfc_lo;
                            bool in_shell = keep && (FULL || d2f > tfc_hi) && d2f < tfs_lo;
                            const bool amb = keep && d2f <= tfs_hi && !in_core && !in_shell;
                            if (__ballot(amb)) {
                                // within 2e-6 of a threshold: the exact integer test decides
                                if (amb) {
                                    const uint64_t d2 = (uint64_t)((int64_t)ddx * ddx) +
                                                        (uint64_t)((int64_t)ddy * ddy) + (uint64_t)((int64_t)ddz * ddz);
                                    in_core = !FULL && d2 <= t_core;
                                    in_shell = !in_core && d2 <= t_shell;
                                }
                            }
                            const uint64_t m_shell = __ballot(in_shell);
                            // positions within the half: members below this lane, minus the
                            // other half's members when this is the upper half
                            const int s_lo = __popc((uint32_t)m_shell);
                            const int s_hi = __popc((uint32_t)(m_shell >> 32));
                            if (in_shell) {
                                const int pos = c.y + lanes_below(m_shell) - (half ? s_lo : 0);
                                if (pos < cap_shell) srow[pos] = (int32_t)sj.w;
                            }
                            c.y += half ? s_hi : s_lo;
                            if (core_row) {
                                const uint64_t m_core = __ballot(in_core);
                                const int c_lo = __popc((uint32_t)m_core);
                                const int c_hi = __popc((uint32_t)(m_core >> 32));
                                if (in_core) {
                                    const int pos = c.x + lanes_below(m_core) - (half ? c_lo : 0);
                                    if (pos < cap_core) crow[pos] = (int32_t)sj.w;
                                }
                                c.x += half ? c_hi : c_lo;
                            }
                        }
                        if (hv && hl == 0) acnt[ka] = c;
                    }
                }
            }
        }
        __syncthreads();
        if (act) {
            const int2 c = acnt[lane];
            ncore[k] = c.x;
            nshell[k] = c.y;
            maxc = max(maxc, c.x);
            maxs = max(maxs, c.y);
        }
        __syncthreads();
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
