// Core and shell lists (Sec. 2.3): C(i) = {j != i : r_ij <= r_core} and
// S(i) = {j : r_core < r_ij <= r_shell}, same-molecule pairs removed, in the
// canonical order "stencil cell offset (dz, dy, dx) lexicographic, then the
// atoms of each cell by id". One traversal of the shell stencil yields both
// lists: the 27 core cells are visited in their own lexicographic order
// inside it. Distances are exact: uint64 squared separations in quanta of
// L / 2^32 against integer thresholds.
//
// Layout: fixed-capacity rows (row k of atom k in cell order), entries are
// cell-sorted atom indices. Counts beyond the capacity are still counted, so
// the host can grow the rows and rebuild.
#include "irbe_device.hpp"
#include "irbe_internal.hpp"

namespace irbe {

__device__ __forceinline__ uint64_t dist2(uint4 a, uint4 b)
{
    const int32_t dx = (int32_t)(b.x - a.x);
    const int32_t dy = (int32_t)(b.y - a.y);
    const int32_t dz = (int32_t)(b.z - a.z);
    return (uint64_t)((int64_t)dx * dx) + (uint64_t)((int64_t)dy * dy) + (uint64_t)((int64_t)dz * dz);
}

__device__ __forceinline__ int wrap(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

template <bool FULL>
__global__ __launch_bounds__(kBlock) void k_build_lists(int64_t n, int n_c, int lo, int hi, uint64_t t_core,
                                                        uint64_t t_shell, const uint4* __restrict__ spos,
                                                        const int32_t* __restrict__ smol,
                                                        const int32_t* __restrict__ cell_start, int cap_core,
                                                        int cap_shell, int32_t* __restrict__ core,
                                                        int32_t* __restrict__ ncore, int32_t* __restrict__ shell,
                                                        int32_t* __restrict__ nshell, int32_t* __restrict__ maxcnt)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint4 si = spos[k];
    const int32_t mi = smol[k];
    const int cx = (int)(((uint64_t)si.x * (uint32_t)n_c) >> 32);
    const int cy = (int)(((uint64_t)si.y * (uint32_t)n_c) >> 32);
    const int cz = (int)(((uint64_t)si.z * (uint32_t)n_c) >> 32);
    const int span = hi - lo + 1;
    const int x0 = wrap(cx + lo, n_c);
    const int len1 = min(span, n_c - x0);
    const int len2 = span - len1;
    int32_t* crow = core + k * (int64_t)cap_core;
    int32_t* srow = shell + k * (int64_t)cap_shell;
    int nc = 0, ns = 0;
    for (int dz = lo; dz <= hi; ++dz) {
        const int z = wrap(cz + dz, n_c);
        for (int dy = lo; dy <= hi; ++dy) {
            const int y = wrap(cy + dy, n_c);
            const int row = (z * n_c + y) * n_c;
            for (int seg = 0; seg < 2; ++seg) {
                const int xa = seg == 0 ? x0 : 0;
                const int xl = seg == 0 ? len1 : len2;
                if (xl <= 0) continue;
                const int jb = cell_start[row + xa];
                const int je = cell_start[row + xa + xl];
                for (int j = jb; j < je; ++j) {
                    const uint4 sj = spos[j];
                    const uint64_t d2 = dist2(si, sj);
                    if (d2 > t_shell || j == (int)k) continue;
                    if (mi >= 0 && smol[j] == mi) continue;
                    if (FULL || d2 > t_core) {
                        if (ns < cap_shell) srow[ns] = j;
                        ++ns;
                    } else {
                        if (nc < cap_core) crow[nc] = j;
                        ++nc;
                    }
                }
            }
        }
    }
    ncore[k] = nc;
    nshell[k] = ns;
    atomicMax(&maxcnt[0], nc);
    atomicMax(&maxcnt[1], ns);
}

hipError_t launch_build_lists(irbe_ctx* h)
{
    const int64_t n = h->cfg.n_atoms;
    const unsigned nb = (unsigned)blocks_for(n, kBlock);
    const Geometry& g = h->geo;
    if (h->full_list)
        k_build_lists<true><<<nb, kBlock, 0, h->stream>>>(n, g.n_c, g.lo, g.hi, g.t_core, g.t_shell, h->spos, h->smol,
                                                          h->cell_start, h->cap_core, h->cap_shell, h->core,
                                                          h->ncore, h->shell, h->nshell, h->maxcnt);
    else
        k_build_lists<false><<<nb, kBlock, 0, h->stream>>>(n, g.n_c, g.lo, g.hi, g.t_core, g.t_shell, h->spos,
                                                           h->smol, h->cell_start, h->cap_core, h->cap_shell, h->core,
                                                           h->ncore, h->shell, h->nshell, h->maxcnt);
    return hipGetLastError();
}

}  // namespace irbe
