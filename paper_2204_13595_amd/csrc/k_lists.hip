// Core and shell lists (Sec. 2.3): C(i) = {j != i : r_ij <= r_core} and
// S(i) = {j : r_core < r_ij <= r_shell}, same-molecule pairs removed, in the
// canonical order "stencil cell offset (dz, dy, dx) lexicographic, then the
// atoms of each cell in cell order (by fixed-point x coordinate, then id)".
// One traversal of the shell stencil yields both lists: the 27 core cells are
// visited in their own lexicographic order inside it. Membership is exact:
// it is that of the uint64 squared separation in quanta of L / 2^32 against
// the integer thresholds.
//
// One wavefront handles the atoms of G consecutive cells of one cell row (one
// lane per atom). For every stencil row (dz, dy) the union of the lanes' x
// ranges is staged in LDS; each lane keeps only the cells its own sphere can
// reach (per-atom pruning of rows and of the x range from exact cell-boundary
// distances; inside the first and last cell of the range, a binary search on
// the x-sorted cell drops the candidates that lie beyond the atom's x
// extent), which leaves the member order unchanged. The atoms whose range is
// not empty are then taken two at a time, one per half-wave: the 32 lanes of
// a half run over the atom's candidates and its members are compacted in
// candidate order.
//
// Candidate test. Every sorted atom has a 16-byte packed record, written once
// per build (k_pack_sorted) and copied into the tile: its fixed-point
// coordinates in units of 2^s quanta taken modulo 2^16 per axis (s is the
// smallest shift at which every separation within a stencil stays below 2^15
// units, so 16-bit differences are exact), the next 5 bits of each coordinate,
// its exclusion id and its index. A packed 16-bit subtraction, a two-term
// integer dot product and a 24-bit multiply give a squared separation d2
// whose components are off by less than delta units each, so d2 below an
// inner bound proves membership and d2 above an outer bound proves
// non-membership. The candidates in between (about one per atom) take a
// second test on the coordinates extended by the 5 extra bits, whose band is
// 32 times narrower; the few left after it take the exact 64-bit test on
// positions read from memory. The LDS footprint (about 6 KB per wavefront)
// leaves room for six or more wavefronts per SIMD. (The lane-per-atom kernel
// for dilute cells below uses the same records.)
//
// Layout: fixed-capacity rows (row k of atom k in cell order), entries are
// cell-sorted atom indices. Counts beyond the capacity are still counted, so
// the host can grow the rows and rebuild; the stores of a pair of atoms go
// through one buffer descriptor that spans just their rows, so an overflowing
// row can only spill into rows that the rebuild rewrites.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "irbe_device.hpp"
#include "irbe_internal.hpp"

namespace irbe {

constexpr int kListWave = 64;
constexpr int kTileCap = 256;  // staged candidates per pass
constexpr int kTilePad = 32;   // slack after the staged candidates for the lanes past a range's end
constexpr int kBufferWord3 = 0x00020000;  // raw buffer descriptor, 32-bit data format
constexpr int kNoStore = 0x7fffffff;      // buffer offset beyond any list descriptor's range

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Integer bounds on an approximate squared separation d2: d2 < *_in proves
// membership of the ball, d2 > *_out proves the opposite. PackedBounds for
// the packed 16-bit coordinates, MidBounds for those extended by e bits.
template <typename T>
struct Bounds {
    T core_in, core_out, shell_in, shell_out, lo_in, lo_out;
};
using PackedBounds = Bounds<uint32_t>;
using MidBounds = Bounds<uint64_t>;

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

// Squared separation of two packed positions (x | y << 16, z): exact in the
// 16-bit units (differences modulo 2^16); the sum of the three squares stays
// below 2^32.
__device__ __forceinline__ uint32_t d2_packed(uint32_t cxy, uint32_t cz, uint32_t axy, uint32_t az)
{
    const s16x2 dxy = __builtin_bit_cast(s16x2, cxy) - __builtin_bit_cast(s16x2, axy);
    const int dz = (short)(cz - az);
    return (uint32_t)__builtin_amdgcn_sdot2(dxy, dxy, dz * dz, false);
}

// Squared separation of two packed positions in units of 2^(s - e) quanta
// from the packed coordinates and their extension bits (x | y << 5 | z << 10
// in the upper half of the z word); each coordinate is then known modulo
// 2^(16 + e) units, its difference is taken in that modulus and is off by less
// than one unit, as the packed test in its own units.
__device__ __forceinline__ uint64_t d2_mid(uint32_t cxy, uint32_t cz, uint32_t axy, uint32_t az, int e)
{
    auto m = [e](uint32_t p, uint32_t x) { return ((p & 0xffffu) << e) | (x & 31u); };
    const int w = 16 - e;
    const int32_t dx = (int32_t)((m(cxy, cz >> 16) - m(axy, az >> 16)) << w) >> w;
    const int32_t dy = (int32_t)((m(cxy >> 16, cz >> 21) - m(axy >> 16, az >> 21)) << w) >> w;
    const int32_t dz = (int32_t)((m(cz, cz >> 26) - m(az, az >> 26)) << w) >> w;
    return (uint64_t)((int64_t)dx * dx) + (uint64_t)((int64_t)dy * dy) + (uint64_t)((int64_t)dz * dz);
}

__device__ __forceinline__ uint64_t dist2_exact(uint4 a, uint4 b)
{
    const int32_t dx = (int32_t)(b.x - a.x);
    const int32_t dy = (int32_t)(b.y - a.y);
    const int32_t dz = (int32_t)(b.z - a.z);
    return (uint64_t)((int64_t)dx * dx) + (uint64_t)((int64_t)dy * dy) + (uint64_t)((int64_t)dz * dz);
}

// Lanes with p set (a wave-uniform mask).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Position of this lane among the set lanes of its half-wave in the mask
// (mlo | mhi << 32), plus base; lowm is all ones in the lower half-wave and
// zero in the upper one, so that the upper lanes skip the lower half's bits.
__device__ __forceinline__ int member_pos(uint32_t mlo, uint32_t mhi, uint32_t lowm, int base)
{
    return (int)__builtin_amdgcn_mbcnt_hi(mhi, __builtin_amdgcn_mbcnt_lo(mlo & lowm, (uint32_t)base));
}

// MODE: split core and shell lists, one full list, the core list alone (the
// shell batch of stencil sampling is drawn from the stencil's cells), or split
// lists with a skin, where S(i) starts at its own threshold t_lo below C(i)'s
// end (the two lists overlap).
enum { kListsSplit = 0, kListsFull = 1, kListsCoreOnly = 2, kListsSplitSkin = 3 };

// The list lengths of atom k: the stored lengths never exceed the row
// capacities, so that every reader stays inside its rows; a longer list sets
// its bit in the error word (the rows then hold its first entries only) and its
// true length still reaches maxcnt, from which the host grows the rows.
template <int MODE>
__device__ __forceinline__ void store_counts(int k, int cc, int cs, int cap_core, int cap_shell,
                                             int32_t* __restrict__ ncore, int32_t* __restrict__ nshell,
                                             uint32_t* __restrict__ err)
{
    if (MODE != kListsFull) {
        ncore[k] = min(cc, cap_core);
        if (cc > cap_core) atomicOr(err, ERR_CORE_CAP);
    } else {
        ncore[k] = cc;
    }
    if (MODE != kListsCoreOnly) {
        nshell[k] = min(cs, cap_shell);
        if (cs > cap_shell) atomicOr(err, ERR_SHELL_CAP);
    }
}

// Wave masks of the lanes in keep that the bounds b settle as members of C(i)
// (mc) and of S(i) (ms), and of those they leave open (amb); each mask is the
// AND of ballots of single compares (scalar operations only).
template <int MODE, bool CORE, typename D>
__device__ __forceinline__ void classify(D d2, const Bounds<D>& b, uint64_t keep, uint64_t& mc, uint64_t& ms,
                                         uint64_t& amb)
{
    if (CORE && MODE == kListsCoreOnly) {
        mc = keep & ballot(d2 < b.core_in);
        ms = 0;
        amb = keep & ~ballot(d2 > b.core_out) & ~mc;
    } else if (CORE && MODE == kListsSplitSkin) {
        const uint64_t b_cin = ballot(d2 < b.core_in), b_lout = ballot(d2 > b.lo_out);
        const uint64_t b_sin = ballot(d2 < b.shell_in);
        mc = keep & b_cin;
        ms = keep & b_lout & b_sin;
        // settled: C(i) either way, and S(i) below t_lo, inside, or beyond t_shell
        const uint64_t set_c = b_cin | ballot(d2 > b.core_out);
        const uint64_t set_s = ballot(d2 < b.lo_in) | (b_lout & b_sin) | ballot(d2 > b.shell_out);
        amb = keep & ~(set_c & set_s);
    } else if (CORE) {
        mc = keep & ballot(d2 < b.core_in);
        ms = keep & ballot(d2 > b.core_out) & ballot(d2 < b.shell_in);
        amb = keep & ~ballot(d2 > b.shell_out) & ~mc & ~ms;
    } else {
        mc = 0;
        ms = keep & ballot(d2 < b.shell_in);
        amb = keep & ~ballot(d2 > b.shell_out) & ~ms;
    }
}

// One chunk per half-wave: this lane's candidate r (k_in: inside the half's
// range) against the half's atom ap (packed x | y, packed z with extension
// bits, exclusion id), atom index k_base + k_rel. The packed bounds settle most
// candidates, the extended coordinates (mid bounds, e bits) nearly all of the
// rest, and the exact test on positions read from memory the few left.
// Members are appended to the half's rows (byte offsets hoff_s, hoff_c within
// the descriptors) after cs and cc, which are advanced; a lane reads its own
// bit of the member masks back for its store. ENC: shell members are stored as
// the 16-bit code `code` (stencil row and candidate position) instead of the
// sorted index.
template <int MODE, bool CORE, bool LAST, bool ENC>
__device__ __forceinline__ void scan_chunk(const u32x4& r, int code, bool k_in, const u32x4& ap, int k_base, int k_rel,
                                           const PackedBounds& tb, const MidBounds& mb, int e, uint64_t t_core,
                                           uint64_t t_lo, uint64_t t_shell, const uint4* __restrict__ spos, int lane,
                                           int hsel, uint32_t lowm, int hoff_s, int hoff_c,
                                           __amdgpu_buffer_rsrc_t rs_s, __amdgpu_buffer_rsrc_t rs_c, int& cs, int& cc)
{
    // (only an atom pair's last chunk holds lanes past the end of a range)
    const uint64_t m_keep = (LAST ? ballot(k_in) : ~0ull) & ballot(r.z != ap.z);
    uint64_t m_core, m_shell, m_amb;
    classify<MODE, CORE>(d2_packed(r.x, r.y, ap.x, ap.y), tb, m_keep, m_core, m_shell, m_amb);
    if (__builtin_expect(m_amb != 0, 0)) {
        // between the packed bounds (wave-uniform branch; the lanes of m_amb
        // take its result)
        // (the atom's operands are copied by an asm statement in this branch, so that
        // the compiler keeps their unpacking, and the copies, here instead of hoisting
        // them to every pair's set-up)
        uint32_t axy, az;
        int ki;
        asm volatile("v_mov_b32 %0, %3\n\tv_mov_b32 %1, %4\n\tv_add_u32 %2, %5, %6"
                     : "=&v"(axy), "=&v"(az), "=&v"(ki)
                     : "v"(ap.x), "v"(ap.y), "s"(k_base), "v"(k_rel));
        uint64_t c2, s2, a2;
        classify<MODE, CORE>(d2_mid(r.x, r.y, axy, az, e), mb, m_amb, c2, s2, a2);
        if (a2 != 0) {
            const bool amb = (a2 >> lane) & 1u;
            const uint64_t d2x = dist2_exact(spos[ki], spos[amb ? (int)r.w : ki]);
            const bool xc = CORE && d2x <= t_core;
            const bool xs = MODE != kListsCoreOnly &&
                            (MODE == kListsSplitSkin ? d2x > t_lo : !xc) && d2x <= t_shell;
            c2 = (c2 & ~a2) | (ballot(xc) & a2);
            s2 = (s2 & ~a2) | (ballot(xs) & a2);
        }
        m_core = (m_core & ~m_amb) | c2;
        m_shell = (m_shell & ~m_amb) | s2;
    }
    if (MODE != kListsCoreOnly) {
        const uint32_t ms_lo = (uint32_t)m_shell, ms_hi = (uint32_t)(m_shell >> 32);
        const int ps_lo = __popc(ms_lo);
        // non-members store past the descriptor's range (dropped)
        const int pos = member_pos(ms_lo, ms_hi, lowm, cs);
        const int off = __builtin_amdgcn_inverse_ballot_w64(m_shell) ? hoff_s + (pos << (ENC ? 1 : 2)) : kNoStore;
        if (ENC) __builtin_amdgcn_raw_buffer_store_b16((uint16_t)code, rs_s, off, 0, 0);
        else __builtin_amdgcn_raw_buffer_store_b32((int)r.w, rs_s, off, 0, 0);
        cs += ps_lo + (hsel & (__popc(ms_hi) - ps_lo));
    }
    if (CORE) {
        const uint32_t mc_lo = (uint32_t)m_core, mc_hi = (uint32_t)(m_core >> 32);
        const int pc_lo = __popc(mc_lo);
        const int pos = member_pos(mc_lo, mc_hi, lowm, cc);
        const int off = __builtin_amdgcn_inverse_ballot_w64(m_core) ? hoff_c + (pos << 2) : kNoStore;
        __builtin_amdgcn_raw_buffer_store_b32((int)r.w, rs_c, off, 0, 0);
        cc += pc_lo + (hsel & (__popc(mc_hi) - pc_lo));
    }
}

template <int MODE, bool ENC>
__global__ __launch_bounds__(kListWave) void k_build_lists_tiled(
    int n_c, int lo, int hi, int G, int prune, int trim, int sh, PackedBounds tb, MidBounds mb, int e, uint64_t t_core,
    uint64_t t_lo, uint64_t t_shell, float tfs_hi, const uint4* __restrict__ spos, const u32x4* __restrict__ spk,
    const int32_t* __restrict__ cell_start, const uint32_t* __restrict__ bound_g, int cap_core, int cap_shell,
    int32_t* __restrict__ core, int32_t* __restrict__ ncore, int32_t* __restrict__ shell,
    int32_t* __restrict__ nshell, int32_t* __restrict__ maxcnt, uint32_t* __restrict__ err, int pb,
    int32_t* __restrict__ sgroup)
{
    __shared__ u32x4 trec[kTileCap + kTilePad];  // candidate: packed x | y, packed z, exclusion id, sorted index
    __shared__ u32x4 apk[kListWave];             // atom: packed x | y, packed z, exclusion id, range start | length << 16
    __shared__ int2 acnt[kListWave];             // atom: core / shell list lengths so far
    int* const cst = reinterpret_cast<int*>(apk);  // a row's cell starts (span_u + 1 <= 4 * kListWave)
    const uint32_t* bound = bound_g;  // indexed by wave-uniform cell coordinates
    const int lane = threadIdx.x;
    const int hl = lane & 31;
    const int hsel = -(lane >> 5);  // all ones in the upper half-wave
    const uint32_t lowm = ~(uint32_t)hsel;
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
        const int na = min(kListWave, a1 - chunk);  // atoms of this chunk
        const uint4 si = act ? spos[k] : make_uint4(0, 0, 0, 0);
        const u32x4 pk = act ? spk[k] : u32x4{0, 0, 0, 0};  // packed x | y, z with extension bits, exclusion id
        const int cx = (int)(((uint64_t)si.x * (uint32_t)n_c) >> 32);
        const int ti = act ? wrap(cx - x0, n_c) : 0;  // lane's home cell in [0, gr)
        // the rows of this chunk's atoms, one buffer descriptor per list: stores of an
        // overflowing row stay within them (and the rebuild that follows rewrites them)
        constexpr int eb = ENC ? 2 : 4;  // bytes per shell entry
        const __amdgpu_buffer_rsrc_t rs_s = __builtin_amdgcn_make_buffer_rsrc(
            (char*)shell + (int64_t)chunk * cap_shell * eb, (short)0, na * cap_shell * eb, kBufferWord3);
        const __amdgpu_buffer_rsrc_t rs_c = __builtin_amdgcn_make_buffer_rsrc(
            core + (int64_t)chunk * cap_core, (short)0, na * cap_core * 4, kBufferWord3);
        acnt[lane] = make_int2(0, 0);
        for (int dz = lo; dz <= hi; ++dz) {
            const int z = wrap(cz + dz, n_c);
            const float gz = prune ? (float)slab_gap(si.z, dz, z, bound) : 0.0f;
            for (int dy = lo; dy <= hi; ++dy) {
                const int y = wrap(cy + dy, n_c);
                const int row = (z * n_c + y) * n_c;
                // rows two or more cells away in y or z hold no core candidate:
                // a whole cell edge (>= the core list radius) lies between them and
                // the atom, and every candidate there lies beyond S(i)'s inner radius
                const bool core_row = MODE != kListsFull && dz >= -1 && dz <= 1 && dy >= -1 && dy <= 1;
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
                        const uint32_t ext = (uint32_t)(__builtin_amdgcn_sqrtf(rem) * 1.000002f) + 2u;
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
                if (ballot(need) == 0) continue;
                // union of the x ranges: segment A (cells xu0 .. xu0+lenA-1), then B (cells 0 ..)
                const int jA = cell_start[row + xu0];
                const int eA = cell_start[row + xu0 + lenA];
                const int lenB = span_u - lenA;
                const int jB = cell_start[row];
                const int eB = lenB > 0 ? cell_start[row + lenB] : jB;
                const int nA = eA - jA;
                const int total = nA + (eB - jB);
                // codes: the row's id above pb bits of candidate position
                const int rcode = ENC ? ((dz - lo) * span_c + (dy - lo)) << pb : 0;
                if (ENC && total > (1 << pb) && lane == 0) atomicOr(err, ERR_SHELL_CODE);
                // lane's range in tile positions: cst[u] = position of the first atom of
                // tile cell u, one lane per cell (cst borrows the atom records' LDS,
                // which the first tile rewrites only after every lane has read it)
                for (int u = lane; u <= span_u; u += kListWave)
                    cst[u] = u < lenA ? cell_start[row + xu0 + u] - jA : nA + cell_start[row + u - lenA] - jB;
                __syncthreads();
                int p_lo = 0, p_hi = 0, pc1 = 0, pc2 = 0;
                if (need) {
                    p_lo = cst[u_lo];
                    p_hi = cst[u_hi + 1];
                    pc1 = u_lo < u_hi ? cst[u_lo + 1] : p_hi;  // end of the first cell
                    pc2 = u_lo < u_hi ? cst[u_hi] : p_lo;      // start of the last cell
                }
                for (int base = 0; base < total; base += kTileCap) {
                    const int cnt = min(kTileCap, total - base);
                    __syncthreads();
                    for (int t = lane; t < cnt; t += kListWave) {
                        const int p = base + t;
                        const int j = p < nA ? jA + p : jB + (p - nA);
                        trec[t] = spk[j];
                    }
                    __syncthreads();
                    if (trim && need && total <= kTileCap) {
                        // the cells are x-sorted, so their packed x is non-decreasing: trim
                        // the first and the last cell of the range of the candidates whose
                        // packed x proves them farther than the sphere's x extent
                        const int ext_u = (int)((uint32_t)ext_i >> sh) + 1;
                        int a = p_lo, b = pc1;
                        while (a < b) {
                            const int m = (a + b) >> 1;
                            if ((int)(short)((trec[m].x - pk.x) & 0xffffu) < -ext_u) a = m + 1;
                            else b = m;
                        }
                        p_lo = a;
                        a = max(pc2, p_lo);
                        b = p_hi;
                        while (a < b) {
                            const int m = (a + b) >> 1;
                            if ((int)(short)((trec[m].x - pk.x) & 0xffffu) <= ext_u) a = m + 1;
                            else b = m;
                        }
                        p_hi = a;
                    }
                    // this tile's part of the lane's range, in tile coordinates
                    const int s0 = need ? max(p_lo, base) - base : 0;
                    const int len_l = need ? max(min(p_hi, base + cnt) - base - s0, 0) : 0;
                    apk[lane] = u32x4{pk.x, pk.y, pk.z, (uint32_t)s0 | ((uint32_t)len_l << 16)};
                    __syncthreads();
                    // atoms are paired with atoms of the same number of 32-candidate
                    // chunks, so no half-wave reads past its own range (+ 31); a lone
                    // atom of a chunk count takes both halves (the upper one idle)
                    const int nch = (len_l + 31) >> 5;
                    uint64_t left = ballot(nch > 0);
                    while (left) {
                        // the chunk counts present, one at a time
                        const int chunks = __builtin_amdgcn_readlane(nch, __builtin_ctzll(left));
                        uint64_t pend = left & ballot(nch == chunks);
                        left &= ~pend;
                        // the pairs of this chunk count; NCH: 1 or 2 chunks (straight-line code), 0
                        // for more (a loop); chosen here once for the chunk count, not per pair
                        auto pairs = [&](auto nch_tag, auto core_tag) {
                            constexpr int NCH = decltype(nch_tag)::value;
                            constexpr bool CORE = decltype(core_tag)::value;
                            while (pend) {
                                // the next two atoms: a in the lower half, b in the upper
                                const int a = __builtin_ctzll(pend);
                                pend &= pend - 1;
                                const bool has_b = pend != 0;
                                const int b = has_b ? __builtin_ctzll(pend) : a;
                                if (has_b) pend &= pend - 1;
                                const int drow = b - a;
                                const int ka = a + (hsel & drow);  // this half's atom
                                const u32x4 ap = apk[ka];
                                const int2 cn = acnt[ka];
                                const int lenm = (int)(ap.w >> 16) - hl;
                                const int qb = (int)(ap.w & 0xffffu) + hl;
                                int cs = cn.y, cc = cn.x;  // this half's atom: list lengths so far
                                // byte offsets of this half's atom's rows in the wave's list rows
                                const int hoff_s = __mul24(ka, cap_shell * eb);
                                // this lane's candidate code in the pair's first chunk
                                const int cq = ENC ? rcode + base + qb : 0;
                                {
                                    const int hoff_c = __mul24(ka, cap_core * 4);
                                    // the two atoms have the same number of chunks: every lane of
                                    // all chunks but the last lies inside its half's range
                                    const int last = NCH == 1 ? 0 : NCH == 2 ? 32 : (chunks - 1) * 32;
                                    if (NCH == 2) {
                                        scan_chunk<MODE, CORE, false, ENC>(trec[qb], cq, true, ap, chunk, ka, tb, mb,
                                                                           e, t_core, t_lo, t_shell, spos, lane, hsel,
                                                                           lowm, hoff_s, hoff_c, rs_s, rs_c, cs, cc);
                                    } else if (NCH == 0) {
                                        int c0 = 0;
                                        do {
                                            scan_chunk<MODE, CORE, false, ENC>(trec[qb + c0], cq + c0, true, ap, chunk,
                                                                               ka, tb, mb, e, t_core, t_lo, t_shell,
                                                                               spos, lane, hsel, lowm, hoff_s, hoff_c,
                                                                               rs_s, rs_c, cs, cc);
                                            c0 += 32;
                                        } while (c0 < last);
                                    }
                                    scan_chunk<MODE, CORE, true, ENC>(trec[qb + last], cq + last, last < lenm, ap,
                                                                      chunk, ka, tb, mb, e, t_core, t_lo, t_shell,
                                                                      spos, lane, hsel, lowm, hoff_s, hoff_c, rs_s,
                                                                      rs_c, cs, cc);
                                }
                                if (lane == 0 || (lane == 32 && has_b)) acnt[ka] = make_int2(cc, cs);
                            }
                        };
                        // (the row's core flag and the chunk count chosen here, once)
                        using one = std::integral_constant<int, 1>;
                        using two = std::integral_constant<int, 2>;
                        using many = std::integral_constant<int, 0>;
                        if (core_row) {
                            if (chunks == 1) pairs(one{}, std::true_type{});
                            else if (chunks == 2) pairs(two{}, std::true_type{});
                            else pairs(many{}, std::true_type{});
                        } else {
                            if (chunks == 1) pairs(one{}, std::false_type{});
                            else if (chunks == 2) pairs(two{}, std::false_type{});
                            else pairs(many{}, std::false_type{});
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (act) {
            const int2 c = acnt[lane];
            store_counts<MODE>(k, c.x, c.y, cap_core, cap_shell, ncore, nshell, err);
            if (ENC) sgroup[k] = g;
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

// ---------------------------------------------------------------------------
// Lane-per-atom form, for dilute systems (a few atoms per cell, e.g. the
// primitive-model electrolytes) with cells narrower than the box
// (2R + 1 <= n_c). The same lists in the same order as k_build_lists_tiled.
// There every atom's range in a stencil row holds only a handful of candidates,
// so a half-wave per atom and row idles most of its lanes; here one wavefront
// takes up to 64 atoms of consecutive cells of one cell row, one atom per lane.
// For every stencil row (dz, dy) the union of the atoms' x ranges is staged in
// LDS as above. The first atom and atom count of every row's union (two index
// ranges at most) are loaded once per group into a table held in registers,
// so that a row's cell starts and the records of its first tile are loaded in
// one memory round trip, issued before the pruning of the rows that follow.
// Each lane computes its own cell range in the union (row pruning) and
// the lanes then walk their ranges in lockstep, lane a testing its k-th
// candidate at step k. A lane appends its shell members (or full-list
// members) to a ring of 8 entries in LDS and every 4 steps the lanes whose
// ring holds 4 unwritten entries store them as one aligned 16-byte segment of
// their list row (at most 3 + 4 entries wait in the ring); core members are
// stored directly. Candidates between the
// packed bounds take the exact test on full positions read from memory (the
// LDS footprint, about 4.4 KB, leaves room for the wavefronts that hide the
// per-row latencies). (In dense cells, such as water's ~13 atoms per cell, the
// lanes' ranges spread over the staged row and the half-wave form is faster.)
// ---------------------------------------------------------------------------
constexpr int kLaneTile = 128;           // staged candidates per pass of a row
constexpr int kRing = 8;                 // ring entries per lane
constexpr int kSeg = 4;                  // entries per stored segment (16 bytes)
constexpr int kRingStride = kRing + 1;   // words per lane's ring (odd: conflict-free lanes)
constexpr double kLaneGroupAtoms = 60.0; // atoms per group the launch aims at (at most 64 per pass)
constexpr double kLaneMaxPerCell = 4.0;  // mean atoms per cell below which the launch takes this form

// A stencil row of the lane-per-atom kernel as loaded: its union's two segments
// (first atom and atoms of A; first atom of B; atoms of both), this lane's raw
// cell start in the union and the records of its first tile.
struct RowLoad {
    int jA, nA, jB, total;
    int cst;
    u32x4 rec[kLaneTile / kListWave];
};

// (eight wavefronts per SIMD requested: the register bound of 64 gains the skin lists 8%, the others are the same)
template <int MODE>
__global__ __launch_bounds__(kListWave, 8) void k_build_lists_lanes(
    int n_c, int lo, int hi, int G, PackedBounds tb, uint64_t t_core, uint64_t t_lo, uint64_t t_shell, float tfs_hi,
    const uint4* __restrict__ spos, const u32x4* __restrict__ spk, const int32_t* __restrict__ cell_start,
    const uint32_t* __restrict__ bound_g,
    int cap_core, int cap_shell, int32_t* __restrict__ core, int32_t* __restrict__ ncore,
    int32_t* __restrict__ shell, int32_t* __restrict__ nshell, int32_t* __restrict__ maxcnt,
    uint32_t* __restrict__ err)
{
    __shared__ u32x4 trec[kLaneTile + 1];          // packed x | y, packed z, exclusion id, sorted index
    __shared__ int32_t ring[kListWave * kRingStride];
    __shared__ int32_t tcs[64];                    // union positions of the row's cells (segment A, then B)
    const uint32_t* bound = bound_g;
    const int lane = threadIdx.x;
    const int span = hi - lo + 1;
    const int groups_per_row = (n_c + G - 1) / G;
    const int g = (int)xcd_block(blockIdx.x, gridDim.x);
    const int rowid = g / groups_per_row;
    const int cz = rowid / n_c, cy = rowid % n_c;
    const int x0 = (g % groups_per_row) * G;
    const int gr = min(G, n_c - x0);
    const int home = (cz * n_c + cy) * n_c;
    const int a0 = cell_start[home + x0], a1 = cell_start[home + x0 + gr];
    const int span_u = gr - 1 + span;           // cells of the union x range
    const int xu0 = wrap(x0 + lo, n_c);         // first cell of the union
    const int lenA = min(span_u, n_c - xu0);    // cells before the wrap
    int32_t* const myring = ring + lane * kRingStride;
    // every stencil row's union: first atom and atom count of segment A (cells
    // xu0 .. xu0 + lenA - 1) and of segment B (cells 0 .. lenB - 1, past the wrap),
    // row ri = (dz, dy) = (lo + ri / span, lo + ri % span) in lane ri % 64 of
    // rtab[ri / 64], loaded once for the group
    const int nrows = span * span;  // at most 2 * kListWave (checked at the launch)
    const int lenB = span_u - lenA;
    int4 rtab[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int ri = h * kListWave + lane;
        rtab[h] = make_int4(0, 0, 0, 0);
        if (ri < nrows) {
            const int row = (wrap(cz + lo + ri / span, n_c) * n_c + wrap(cy + lo + ri % span, n_c)) * n_c;
            const int ja = cell_start[row + xu0], jb = cell_start[row];
            rtab[h] = make_int4(ja, cell_start[row + xu0 + lenA] - ja, jb, lenB > 0 ? cell_start[row + lenB] - jb : 0);
        }
    }
    // a row's union from the table, this lane's cell start in it and the records of
    // its first tile, issued together (one memory round trip)
    // first and last coordinates of the stencil's z and y cell slabs, lane l for the
    // offset lo + l (span <= 11 here), read back with readlane
    const int ls = min(lane, span - 1);
    const int zs = wrap(cz + lo + ls, n_c), ys = wrap(cy + lo + ls, n_c);
    const uint32_t zlo = bound[zs], zhi = bound[zs + 1] - 1u, ylo = bound[ys], yhi = bound[ys + 1] - 1u;
    // distance from coordinate s to the slab at offset d (as slab_gap)
    auto gap = [](uint32_t s, int d, uint32_t lo_t, uint32_t hi_t, int idx) __attribute__((always_inline)) {
        if (d > 0) return (uint32_t)__builtin_amdgcn_readlane((int)lo_t, idx) - s;
        if (d < 0) return s - (uint32_t)__builtin_amdgcn_readlane((int)hi_t, idx);
        return 0u;
    };
    // the row after (dz, dy) in the stencil's lexicographic order
    auto step_row = [&](int& dz, int& dy) __attribute__((always_inline)) {
        if (++dy > hi) {
            dy = lo;
            ++dz;
        }
    };
    auto row_load = [&](int ri, int dz, int dy) __attribute__((always_inline)) {
        RowLoad d;
        const int h = ri >> 6, rl = ri & (kListWave - 1);
        d.jA = __builtin_amdgcn_readlane(h ? rtab[1].x : rtab[0].x, rl);
        d.nA = __builtin_amdgcn_readlane(h ? rtab[1].y : rtab[0].y, rl);
        d.jB = __builtin_amdgcn_readlane(h ? rtab[1].z : rtab[0].z, rl);
        d.total = d.nA + __builtin_amdgcn_readlane(h ? rtab[1].w : rtab[0].w, rl);
        const int row = (wrap(cz + dz, n_c) * n_c + wrap(cy + dy, n_c)) * n_c;
        // (every lane loads, from an index inside the arrays, so that no load sits
        // in a branch and the waits for these registers can be counted exactly;
        // lanes past the union or the tile do not use theirs)
        const int lc = min(lane, span_u);
        d.cst = cell_start[lc < lenA ? row + xu0 + lc : row + lc - lenA];
        const int cnt0 = min(kLaneTile, d.total);
#pragma unroll
        for (int q = 0; q < kLaneTile / kListWave; ++q) {
            const int t = q * kListWave + lane;
            d.rec[q] = spk[t < cnt0 ? (t < d.nA ? d.jA + t : d.jB + (t - d.nA)) : a0];
        }
        return d;
    };
    int maxc = 0, maxs = 0;
    for (int chunk = a0; chunk < a1; chunk += kListWave) {
        const int k = chunk + lane;
        const bool act = k < a1;
        const uint4 si = act ? spos[k] : make_uint4(0, 0, 0, 0);
        const int cx = (int)(((uint64_t)si.x * (uint32_t)n_c) >> 32);
        const int ti = act ? wrap(cx - x0, n_c) : 0;  // lane's home cell in [0, gr)
        const u32x4 pk = act ? spk[k] : u32x4{0, 0, 0, 0};  // packed x | y, z, exclusion id
        const uint32_t axy = pk.x, az = pk.y, amol = pk.z;
        int32_t* const crow = core + (int64_t)k * cap_core;
        int32_t* const srow = shell + (int64_t)k * cap_shell;
        int cc = 0, cs = 0;  // list lengths so far
        int fs = 0;          // shell entries already stored (a multiple of kSeg)
        // the lane's range in row ri = (dz, dy): cells [u_lo, u_hi] of the union, pruned by
        // the row gap; the first row at or after ri that some lane needs (nrows: none),
        // with (dz, dy) advanced to it
        auto next_row = [&](int ri, int& dz, int& dy, int& u_lo, int& u_hi, bool& need)
                            __attribute__((always_inline)) -> int {
            for (; ri < nrows; ++ri, step_row(dz, dy)) {
                if (MODE == kListsCoreOnly && (dz < -1 || dz > 1 || dy < -1 || dy > 1)) continue;
                u_lo = ti;
                u_hi = ti + span - 1;
                need = act;
                if (act) {
                    const float gz = (float)gap(si.z, dz, zlo, zhi, dz - lo);
                    const float gy = (float)gap(si.y, dy, ylo, yhi, dy - lo);
                    const float rem = tfs_hi - gy * gy - gz * gz;
                    if (rem < 0.0f) {
                        need = false;
                    } else {
                        const uint32_t ext = (uint32_t)(__builtin_amdgcn_sqrtf(rem) * 1.000002f) + 2u;
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
                if (ballot(need) != 0) return ri;
            }
            return nrows;
        };
        int u_lo = 0, u_hi = 0;
        bool need = false;
        int dz = lo, dy = lo;
        int rc = next_row(0, dz, dy, u_lo, u_hi, need);
        while (rc < nrows) {
            // the row's loads are in flight while the next needed row is found
            const RowLoad cur = row_load(rc, dz, dy);
            int u_lo_n = 0, u_hi_n = 0;
            bool need_n = false;
            int dz_n = dz, dy_n = dy;
            step_row(dz_n, dy_n);
            const int rn = next_row(rc + 1, dz_n, dy_n, u_lo_n, u_hi_n, need_n);
            const bool core_row = MODE != kListsFull && dz >= -1 && dz <= 1 && dy >= -1 && dy <= 1;
            const int jA = cur.jA, nA = cur.nA, jB = cur.jB, total = cur.total;
            // (LDS accesses of the one wavefront of the workgroup take effect in
            // order: the previous row's reads precede these writes)
            if (lane <= span_u) tcs[lane] = cur.cst - (lane < lenA ? jA : jB - nA);
#pragma unroll
            for (int h = 0; h < kLaneTile / kListWave; ++h)
                if (h * kListWave + lane < min(kLaneTile, total)) trec[h * kListWave + lane] = cur.rec[h];
            asm volatile("" ::: "memory");
            const int p_lo = need ? tcs[u_lo] : 0;
            const int p_hi = need ? tcs[u_hi + 1] : 0;
            for (int base = 0; base < total; base += kLaneTile) {
                const int cnt = min(kLaneTile, total - base);
                if (base > 0) {
                    // a row longer than one tile (crowded cells): its later tiles
                    __syncthreads();
                    for (int t = lane; t < cnt; t += kListWave) {
                        const int p = base + t;
                        const int j = p < nA ? jA + p : jB + (p - nA);
                        trec[t] = spk[j];
                    }
                    __syncthreads();
                }
                // this tile's part of the range, in tile positions
                const int s0 = need ? max(p_lo, base) - base : 0;
                const int len = need ? max(min(p_hi, base + cnt) - base - s0, 0) : 0;
                int steps = len;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) steps = max(steps, __shfl_xor(steps, off, 64));
                steps = __builtin_amdgcn_readfirstlane(steps);  // (every lane holds the maximum)
                for (int st = 0; st < steps; ++st) {
                    const bool k_in = st < len;
                    const int tp = k_in ? s0 + st : kLaneTile;
                    const u32x4 r = trec[tp];
                    const uint32_t d2 = d2_packed(r.x, r.y, axy, az);
                    const bool keep = k_in && r.z != amol;
                    bool in_core = false, in_shell = false, amb;
                    if (MODE == kListsCoreOnly) {
                        in_core = keep && d2 < tb.core_in;
                        amb = keep && !in_core && d2 <= tb.core_out;
                    } else if (MODE == kListsSplitSkin) {
                        const bool c_in = d2 < tb.core_in, c_out = d2 > tb.core_out;
                        const bool l_in = d2 < tb.lo_in, l_out = d2 > tb.lo_out;
                        const bool s_in = d2 < tb.shell_in, s_out = d2 > tb.shell_out;
                        in_core = keep && c_in;
                        in_shell = keep && l_out && s_in;
                        amb = keep && !((c_in || c_out) && (l_in || (l_out && s_in) || s_out));
                    } else if (MODE == kListsSplit) {
                        const bool c_in = d2 < tb.core_in, c_out = d2 > tb.core_out;
                        const bool s_in = d2 < tb.shell_in, s_out = d2 > tb.shell_out;
                        in_core = keep && c_in;
                        in_shell = keep && c_out && s_in;
                        amb = keep && !c_in && !in_shell && !s_out;
                    } else {
                        in_shell = keep && d2 < tb.shell_in;
                        amb = keep && !in_shell && d2 <= tb.shell_out;
                    }
                    if (amb) {
                        // between the bounds: the exact test on full positions decides
                        const uint4 sj = spos[(int)r.w];
                        const int32_t dx = (int32_t)(sj.x - si.x);
                        const int32_t dy2 = (int32_t)(sj.y - si.y);
                        const int32_t dz2 = (int32_t)(sj.z - si.z);
                        const uint64_t d2x = (uint64_t)((int64_t)dx * dx) + (uint64_t)((int64_t)dy2 * dy2) +
                                             (uint64_t)((int64_t)dz2 * dz2);
                        in_core = MODE != kListsFull && d2x <= t_core;
                        in_shell = MODE != kListsCoreOnly &&
                                   (MODE == kListsSplitSkin ? d2x > t_lo : !in_core) && d2x <= t_shell;
                    }
                    if (MODE != kListsCoreOnly && in_shell) {
                        myring[cs & (kRing - 1)] = (int32_t)r.w;
                        ++cs;
                    }
                    if (MODE != kListsFull && core_row && in_core) {
                        if (cc < cap_core) crow[cc] = (int32_t)r.w;
                        ++cc;
                    }
                    if (MODE != kListsCoreOnly && (st & (kSeg - 1)) == kSeg - 1) {
                        // lanes with a full segment store it (at most one per kSeg steps)
                        if (cs - fs >= kSeg) {
                            const int o = fs & (kRing - 1);
                            if (fs + kSeg <= cap_shell)
                                *(int4*)(srow + fs) = make_int4(myring[o], myring[o + 1], myring[o + 2], myring[o + 3]);
                            fs += kSeg;
                        }
                    }
                }
                if (MODE != kListsCoreOnly) {
                    // at most one full segment waits after the last step
                    if (cs - fs >= kSeg) {
                        const int o = fs & (kRing - 1);
                        if (fs + kSeg <= cap_shell)
                            *(int4*)(srow + fs) = make_int4(myring[o], myring[o + 1], myring[o + 2], myring[o + 3]);
                        fs += kSeg;
                    }
                }
            }
            rc = rn;
            dz = dz_n;
            dy = dy_n;
            u_lo = u_lo_n;
            u_hi = u_hi_n;
            need = need_n;
        }
        if (MODE != kListsCoreOnly) {
            // the last, partial segment
            for (int e = fs; e < cs; ++e)
                if (e < cap_shell) srow[e] = myring[e & (kRing - 1)];
        }
        if (act) {
            store_counts<MODE>(k, cc, cs, cap_core, cap_shell, ncore, nshell, err);
            maxc = max(maxc, cc);
            maxs = max(maxs, cs);
        }
        __syncthreads();
    }
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

// Stencil sampling: |K(i)|, the number of atoms in the shell stencil's cells
// around atom i's cell (span^2 rows of span cells, each row at most two index
// ranges of the cell-sorted atoms), written as the shell count of every atom
// of the cell together with the cell itself (the build-time cell, which the
// batch decode uses even after the atoms have moved); one thread per cell, and
// the largest count raises maxcnt[1].
__global__ __launch_bounds__(kBlock) void k_stencil_counts(int n_c, int lo, int span,
                                                           const int32_t* __restrict__ cell_start,
                                                           int32_t* __restrict__ nshell, int32_t* __restrict__ scell,
                                                           int32_t* __restrict__ maxcnt, uint32_t* __restrict__ err)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cells = (int64_t)n_c * n_c * n_c;
    int m = 0;
    if (c < cells) {
        const int cx = (int)(c % n_c), cy = (int)((c / n_c) % n_c), cz = (int)(c / ((int64_t)n_c * n_c));
        const int x0 = wrap(cx + lo, n_c);
        const int la = min(span, n_c - x0);  // cells before the wrap
        for (int dz = 0; dz < span; ++dz) {
            const int z = wrap(cz + lo + dz, n_c);
            for (int dy = 0; dy < span; ++dy) {
                const int row = (z * n_c + wrap(cy + lo + dy, n_c)) * n_c;
                m += cell_start[row + x0 + la] - cell_start[row + x0];
                if (span > la) m += cell_start[row + span - la] - cell_start[row];
            }
        }
        // the batch ranks are 16-bit: a larger stencil is an error (and its count is clamped)
        if (m > 65535) atomicOr(err, ERR_SHELL_CAP);
        for (int k = cell_start[c]; k < cell_start[c + 1]; ++k) {
            nshell[k] = min(m, 65535);
            scell[k] = (int32_t)c;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(&maxcnt[1], m);
}

// Packed records of the sorted atoms for k_build_lists_tiled: x | y << 16 and
// z, each fixed-point coordinate in units of 2^sh quanta taken modulo 2^16
// (the separations within a stencil stay below 2^15 units, so their 16-bit
// differences are exact), the next e bits of the three coordinates
// (x | y << 5 | z << 10) in the upper half of the z word, the exclusion id
// (molecule, or -2 - k for an atom without one) and the sorted index k.
__global__ __launch_bounds__(kBlock) void k_pack_sorted(int64_t n, int sh, int e, const uint4* __restrict__ spos,
                                                       const int32_t* __restrict__ smol, u32x4* __restrict__ spk)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint4 s = spos[k];
    const int32_t m = smol[k];
    const uint32_t mk = (1u << e) - 1u;
    const int se = sh - e;
    const uint32_t ext = ((s.x >> se) & mk) | (((s.y >> se) & mk) << 5) | (((s.z >> se) & mk) << 10);
    spk[k] = u32x4{((s.x >> sh) & 0xffffu) | ((s.y >> sh) << 16), ((s.z >> sh) & 0xffffu) | (ext << 16),
                   (uint32_t)(m >= 0 ? m : -2 - (int32_t)k), (uint32_t)k};
}

namespace {

// Shift s and bounds of the packed candidate test. With a pruned stencil
// every separation a lane tests (an atom and a candidate of its own stencil)
// lies within R + 1 cell edges (+ rounding) per axis; s is the smallest shift
// that fits that in 16 signed bits with two units to spare, so the 16-bit
// differences of the packed global coordinates are exact modulo 2^16, and each
// packed component is off by less than delta = 1 unit. When
// the stencil wraps the box, the top 16 bits of the coordinates are used
// (s = 16, modular differences, delta = 3).
// With e = sum of component errors: D <= d2 + 2 delta sqrt(3 d2) + 3 delta^2
// and D >= d2 - 2 delta sqrt(3 d2) for the exact squared separation D in the
// same units; the bounds follow, with one unit of margin for rounding here.
// The mid test extends each packed coordinate by the next e = min(s, 5) bits
// (units of 2^(s - e) quanta, delta = 1, differences that no longer wrap);
// without pruning it is switched off (every candidate stays open for the
// exact test).
struct PackedGeometry {
    int sh = 16;
    PackedBounds tb{};
    MidBounds mb{};
    int e = 0;
};

PackedGeometry packed_geometry(const Geometry& g, bool prune)
{
    PackedGeometry p;
    const double E = 4294967296.0 / (double)g.n_c;
    double delta = 3.0;
    if (prune) {
        const double M = (g.reach + 1.0) * E + 4.0;
        for (int s = 0; s <= 15; ++s) {
            if (M <= std::ldexp(1.0, 15 + s) - std::ldexp(1.0, s + 1)) {
                p.sh = s;
                delta = 1.0;
                break;
            }
        }
    }
    // bounds in units of 2^s quanta (component errors below delta units), as doubles
    auto inner = [](uint64_t t, int s, double delta) -> double {
        const double T = (double)t / std::ldexp(1.0, 2 * s);
        const double v = std::floor(T - 2.0 * delta * std::sqrt(3.0 * T) - 3.0 * delta * delta - 1.0);
        return v > 0.0 ? v : 0.0;
    };
    auto outer = [](uint64_t t, int s, double delta) -> double {
        const double T = (double)t / std::ldexp(1.0, 2 * s);
        const double r = delta * std::sqrt(3.0) + std::sqrt(3.0 * delta * delta + T);
        double o = std::ceil(r * r) + 2.0;
        while ((o + 1.0) - 2.0 * delta * std::sqrt(3.0 * (o + 1.0)) <= T + 1.0) o += 1.0;
        return o;
    };
    auto u32 = [](double v) { return v < 4294967295.0 ? (uint32_t)v : 4294967295u; };
    p.tb.core_in = u32(inner(g.tl_core, p.sh, delta));
    p.tb.core_out = u32(outer(g.tl_core, p.sh, delta));
    p.tb.shell_in = u32(inner(g.tl_shell, p.sh, delta));
    p.tb.shell_out = u32(outer(g.tl_shell, p.sh, delta));
    p.tb.lo_in = u32(inner(g.tl_lo, p.sh, delta));
    p.tb.lo_out = u32(outer(g.tl_lo, p.sh, delta));
    if (prune && p.sh < 16) {
        p.e = std::min(p.sh, 5);
        const int s = p.sh - p.e;
        auto u64 = [](double v) { return v < 1.8e19 ? (uint64_t)v : ~0ull; };
        p.mb.core_in = u64(inner(g.tl_core, s, 1.0));
        p.mb.core_out = u64(outer(g.tl_core, s, 1.0));
        p.mb.shell_in = u64(inner(g.tl_shell, s, 1.0));
        p.mb.shell_out = u64(outer(g.tl_shell, s, 1.0));
        p.mb.lo_in = u64(inner(g.tl_lo, s, 1.0));
        p.mb.lo_out = u64(outer(g.tl_lo, s, 1.0));
    } else {
        p.e = 0;
        p.mb = MidBounds{0, ~0ull, 0, ~0ull, 0, ~0ull};
    }
    return p;
}

}  // namespace

bool shell16_possible(const irbe_ctx* h)
{
    const Geometry& g = h->geo;
    if (h->full_list || h->stencil) return false;
    const bool narrow = 2 * g.reach + 1 <= g.n_c;
    const int span = g.hi - g.lo + 1;
    const double per_cell = (double)h->cfg.n_atoms / (double)g.n_cells;
    const bool lanes = narrow && per_cell < kLaneMaxPerCell && span * span <= 2 * kListWave;
    return narrow && !lanes && span * span <= 64;
}

hipError_t launch_build_lists(irbe_ctx* h)
{
    Geometry g = h->geo;
    if (h->stencil) {
        // core list only: the core stencil, and rows pruned by the core radius
        g.reach = 1;
        g.lo = -1;
        g.hi = 1;
    }
    const int n_c = g.n_c;
    const bool narrow = 2 * g.reach + 1 <= n_c;
    // cells per wavefront (measured optima): about 40 atoms for the split and full
    // lists (3 cells of water), about 76 for the core list alone (6 cells of water,
    // two passes of 64 lanes: its 9 short stencil rows make the per-row set-up the
    // larger cost), more cells in sparse systems such as the electrolytes with
    // about one atom per cell; the union x range of the group's stencils within one
    // period of the box, and the groups of a cell row balanced (a short last group
    // leaves its wavefront mostly idle)
    const double per_cell = (double)h->cfg.n_atoms / (double)g.n_cells;
    // dilute cells take the lane-per-atom kernel (up to 64 atoms per pass of its
    // wavefront, its groups aiming at kLaneGroupAtoms)
    const int span = g.hi - g.lo + 1;
    const bool lanes = narrow && per_cell < kLaneMaxPerCell && span * span <= 2 * kListWave;
    const double g_atoms = lanes ? kLaneGroupAtoms : (h->stencil ? 76.0 : 40.0);
    const double g_min = lanes ? 1.0 : (h->stencil ? 6.0 : 3.0);
    const int g_want = (int)std::lround(std::min(64.0, std::max(g_min, g_atoms / std::max(per_cell, 0.75))));
    int g_cap = narrow ? std::max(1, std::min(g_want, n_c - 2 * g.reach)) : 1;
    // the lane-per-atom kernel keeps the union's cell starts in 64 LDS words
    if (lanes) g_cap = std::min(g_cap, 64 - (g.hi - g.lo + 1));
    // the tiled kernel keeps a row's G - 1 + (2R + 1) + 1 cell starts in 4 * 64 LDS words
    else g_cap = std::min(g_cap, 4 * kListWave - (g.hi - g.lo + 1));
    const int groups_per_row = (n_c + g_cap - 1) / g_cap;
    const int G = (n_c + groups_per_row - 1) / groups_per_row;
    const int prune = narrow ? 1 : 0;
    const int64_t groups = (int64_t)n_c * n_c * ((n_c + G - 1) / G);
    const PackedGeometry pg = packed_geometry(g, narrow);
    // packed x is monotone along a cell only when no relative coordinate wraps
    const int trim = narrow && pg.sh < 16 ? 1 : 0;
    // FP32 threshold of the outermost list with a relative margin of 2e-6, far
    // above the FP32 rounding of the row gaps: the row pruning never drops a member.
    const float tf_hi = (float)(h->stencil ? g.tl_core : g.tl_shell) * 1.000002f;
    // 16-bit shell entries, when the rows were allocated for them: split lists of
    // the tiled build over a stencil of at most 64 rows (a row id of rbits bits,
    // pb bits of candidate position)
    const int nrows = span * span;
    const int rbits = nrows > 1 ? 32 - __builtin_clz((unsigned)(nrows - 1)) : 0;
    const int pb = 16 - rbits;
    const bool enc = h->shell_bytes == 2;
    if (enc && (lanes || !narrow || h->full_list || h->stencil || h->sgroup == nullptr || nrows > 64))
        return hipErrorInvalidValue;
    h->shell16 = enc;
    h->lcode = enc ? ListCode{h->cell_start, h->sgroup, n_c, g.lo, span, G, (n_c + G - 1) / G, pb} : ListCode{};
#define IRBE_LISTS_ARGS                                                                                           \
    n_c, g.lo, g.hi, G, prune, trim, pg.sh, pg.tb, pg.mb, pg.e, g.tl_core, g.tl_lo, g.tl_shell, tf_hi, h->spos,      \
        (const u32x4*)h->spk, h->cell_start, h->cell_bound, h->cap_core, h->cap_shell, h->core, h->ncore, h->shell,  \
        h->nshell, h->maxcnt, h->err, pb, h->sgroup
#define IRBE_LANES_ARGS                                                                                            \
    n_c, g.lo, g.hi, G, pl.tb, g.tl_core, g.tl_lo, g.tl_shell, tf_hi, h->spos, (const u32x4*)h->spk, h->cell_start, \
        h->cell_bound, h->cap_core, h->cap_shell, h->core, h->ncore, h->shell, h->nshell, h->maxcnt, h->err
    if (lanes) {
        // the packed records as for one cell per group: only a lane's own candidates
        // (within the stencil of its cell) are tested, so 16-bit differences of the
        // global coordinates are exact
        const PackedGeometry pl = packed_geometry(g, true);
        k_pack_sorted<<<(unsigned)blocks_for(h->cfg.n_atoms, kBlock), kBlock, 0, h->stream>>>(
            h->cfg.n_atoms, pl.sh, pl.e, h->spos, h->smol, (u32x4*)h->spk);
        if (h->full_list)
            k_build_lists_lanes<kListsFull><<<(unsigned)groups, kListWave, 0, h->stream>>>(IRBE_LANES_ARGS);
        else if (h->stencil)
            k_build_lists_lanes<kListsCoreOnly><<<(unsigned)groups, kListWave, 0, h->stream>>>(IRBE_LANES_ARGS);
        else if (g.skin)
            k_build_lists_lanes<kListsSplitSkin><<<(unsigned)groups, kListWave, 0, h->stream>>>(IRBE_LANES_ARGS);
        else
            k_build_lists_lanes<kListsSplit><<<(unsigned)groups, kListWave, 0, h->stream>>>(IRBE_LANES_ARGS);
    } else {
        k_pack_sorted<<<(unsigned)blocks_for(h->cfg.n_atoms, kBlock), kBlock, 0, h->stream>>>(
            h->cfg.n_atoms, pg.sh, pg.e, h->spos, h->smol, (u32x4*)h->spk);
        if (h->full_list)
            k_build_lists_tiled<kListsFull, false><<<(unsigned)groups, kListWave, 0, h->stream>>>(IRBE_LISTS_ARGS);
        else if (h->stencil)
            k_build_lists_tiled<kListsCoreOnly, false><<<(unsigned)groups, kListWave, 0, h->stream>>>(IRBE_LISTS_ARGS);
        else if (g.skin && enc)
            k_build_lists_tiled<kListsSplitSkin, true><<<(unsigned)groups, kListWave, 0, h->stream>>>(IRBE_LISTS_ARGS);
        else if (g.skin)
            k_build_lists_tiled<kListsSplitSkin, false><<<(unsigned)groups, kListWave, 0, h->stream>>>(IRBE_LISTS_ARGS);
        else if (enc)
            k_build_lists_tiled<kListsSplit, true><<<(unsigned)groups, kListWave, 0, h->stream>>>(IRBE_LISTS_ARGS);
        else
            k_build_lists_tiled<kListsSplit, false><<<(unsigned)groups, kListWave, 0, h->stream>>>(IRBE_LISTS_ARGS);
    }
#undef IRBE_LANES_ARGS
#undef IRBE_LISTS_ARGS
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !h->stencil) return e;
    // stencil sampling: |K(i)| (the atoms of the shell stencil's cells) as the shell count
    const Geometry& gs = h->geo;
    const int64_t cells = gs.n_cells;
    k_stencil_counts<<<(unsigned)blocks_for(cells, kBlock), kBlock, 0, h->stream>>>(
        gs.n_c, gs.lo, gs.hi - gs.lo + 1, h->cell_start, h->nshell, h->scell, h->maxcnt, h->err);
    return hipGetLastError();
}

}  // namespace irbe
