// Internal declarations of the HIP implementation: the handle, the launch
// helpers and the kernel entry points shared between the translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "irbe.h"

namespace irbe {

// Error-word bits set by kernels and read back at the next waiting call.
enum : uint32_t { ERR_NONFINITE = 1u, ERR_CORE_CAP = 2u, ERR_SHELL_CAP = 4u, ERR_SHELL_CODE = 8u };

// 16-bit shell entries. The list build treats the cells of a cell row in groups
// of G consecutive cells (the last group of a row may be shorter); for stencil
// row (dz, dy) a group's candidates are the atoms of the union of its cells'
// x ranges in that row, at most two index ranges of the sorted atoms (the
// second after the periodic wrap). An entry stores the row's id
// (dz - lo) * span + (dy - lo) in its high bits and the member's position in
// that candidate range in its low pb bits; the member is then
// a + p for p < na, else b + (p - na), with a, na the first atom and length of
// the first range and b the first atom of the second.
struct ListCode {
    const int32_t* cell_start;  // [n_c^3 + 1] of the build
    const int32_t* sgroup;      // [N] list-build group of each sorted atom
    int n_c, lo, span, G, gpr, pb;  // gpr: groups per cell row
};

constexpr int kBlock = 256;          // threads per block of the per-atom kernels
constexpr int kReduceBlock = 256;    // threads of the deterministic final reductions
constexpr int kPairPartials = 16;    // FP64 values per block of the pair kernel
constexpr int kRhoAtomsPerThread = 8;  // fewest atoms per thread of the structure-factor kernels
constexpr int kMaxTypesGrad = 4;     // LJ parameter gradients: n_types <= 4
// atoms per wavefront in the cooperative pair kernels: the adjoint, the forward
// kernel with list-drawn batches, and the forward kernel with stencil sampling
constexpr int kAtomsPerWave = 8;
constexpr int kAtomsPerWaveList = 4;   // full lists
constexpr int kAtomsPerWaveSplit = 8;  // split lists (the optimum with 16-bit shell entries; the same with
                                       // 32-bit ones, so that the per-block sums and results do not change)
constexpr int kAtomsPerWaveStencil = 16;
// Shell-adjoint transpose: scatter records staged per block in LDS, then
// bucketed by destination cell row (y, z) and reduced per row.
constexpr int kBucketRowLds = 2048;  // atoms of a row accumulated in LDS (the rest: device atomics)
constexpr int kBucketRecF = 1200;    // staged records per block (budget), FP32
constexpr int kBucketRecD = 600;     // staged records per block (budget), FP64
constexpr int kBucketRecMaxF = 2048; // staged records per block (LDS limit), FP32
constexpr int kBucketRecMaxD = 1024; // staged records per block (LDS limit), FP64
constexpr int kBucketMaxKeys = 256;  // (source row, destination row) keys per block
constexpr int kBucketSlack = 64;     // records of spare capacity per destination row

// Per-k constants of the force kernels: k (3), then coefficient products.
template <typename real>
struct KForce {
    real kx, ky, kz;
    real a;  // ke c_l Im(rho_l)
    real b;  // ke c_l Re(rho_l)
    real pad0, pad1, pad2;
};

template <typename real>
struct KAdj {
    real kx, ky, kz;
    real ar, ai;  // ke c_l A_l
    real rr, ri;  // ke c_l rho_l
    real pad;
};

// LJ pair table entry: force 48 eps s^12, 24 eps s^6; energy 4 eps s^12, 4 eps s^6;
// the term acts at r^2 < rc2 (the largest finite value without a cutoff) and its
// energy is lowered by esh there (the shifted-truncated form).
template <typename real>
struct LJ {
    real a12, b6, c12, c6, rc2, esh;
};

struct Geometry {
    int32_t n_c = 0;
    int32_t reach = 0;      // R: shell stencil half-width in cells
    int32_t lo = 0, hi = 0; // shell stencil offsets per axis, inclusive
    uint64_t t_core = 0, t_shell = 0;  // membership at force time: r <= r_core, r <= r_shell
    // list thresholds: C(i) D^2 <= tl_core, S(i) tl_lo < D^2 <= tl_shell (the
    // above without a skin; with one, r_core + skin, r_core - skin, r_shell + skin)
    uint64_t tl_core = 0, tl_lo = 0, tl_shell = 0;
    bool skin = false;      // lists built with a skin: entries tested at force time
    double inv_l = 0.0;
    double quantum = 0.0;   // L / 2^32
    int64_t n_cells = 0;
};

}  // namespace irbe

struct irbe_ctx {
    irbe_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    bool fp64 = false;
    bool full_list = false;
    bool stencil = false;             // shell batch drawn from the stencil's cells (no shell list)
    size_t real_size = 4;
    irbe::Geometry geo;
    std::string last_error;

    // k table
    int32_t kM = 0;
    double kH = 0.0, kS = 0.0;

    // state
    bool have_system = false;
    bool have_lists = false;
    int32_t cap_core = 0, cap_shell = 0;
    // longest core / shell (or stencil) list of the last build whose lengths the
    // host has seen: exact after a waiting build, possibly stale after the
    // asynchronous ones (which only read them back when they have completed), so
    // only choices of speed use them; sizes that must hold every list use
    // shell_bound()
    int32_t max_core = 0, max_shell = 0;
    bool lists_sized = false;         // a waiting build has sized the list rows
    int32_t* chk_host = nullptr;      // pinned [3]: error word, max core, max shell of the last build
    hipEvent_t chk_event = nullptr;   // recorded after the copy into chk_host
    bool chk_pending = false;         // chk_host awaits a completed copy
    // Upper bound on every atom's shell (or full, or stencil) list length.
    int32_t shell_bound() const { return stencil ? max_shell : cap_shell; }
    uint64_t last_force_step = 0;
    bool have_force_step = false;
    std::vector<double> lj_sigma_host, lj_eps_host;

    // device memory, all owned by the handle
    uint32_t* err = nullptr;          // error word
    int32_t* maxcnt = nullptr;        // [2] max core / shell count of the last build
    uint64_t* ktab = nullptr;         // [2M+1]
    void* q_orig = nullptr;           // real[N]
    int32_t* type_orig = nullptr;     // [N]
    int32_t* mol_orig = nullptr;      // [N]
    void* lj = nullptr;               // LJ<real>[n_t^2]
    void* lj_raw = nullptr;           // real[2 n_t^2]: sigma, eps
    int32_t* xoff = nullptr;          // [N+1] exclusion partners per atom (caller ids)
    int32_t* xidx = nullptr;
    int32_t* sxidx = nullptr;         // [n_excl] xidx entries as sorted indices (rebuilt with the cells)
    int2* sxr = nullptr;              // [N] sorted atom's range (first, count) in sxidx
    int64_t n_excl = 0;
    double* sumq2 = nullptr;          // [1]
    double* q2part = nullptr;

    uint4* sq = nullptr;              // [N] quantized position + cell, caller order
    int32_t* cell_count = nullptr;    // [n_cells]
    int32_t* cell_start = nullptr;    // [n_cells + 1]
    uint32_t* cell_bound = nullptr;   // [n_c + 1] first fixed-point coordinate of each cell row/column
    std::vector<int32_t*> scan_levels;
    std::vector<int64_t> scan_sizes;
    int32_t* perm = nullptr;          // [N] sorted -> caller id
    int32_t* rank = nullptr;          // [N] caller id -> sorted
    uint4* spos = nullptr;            // [N] sorted {sx, sy, sz, type}
    uint4* spk = nullptr;             // [N] sorted packed records of the list build
    int32_t* brow = nullptr;          // [N] cell (z << 16 | y) at the build of each sorted atom (lists with a skin)
    uint4* spq = nullptr;             // [N] sorted {sx, sy, sz, FP32 charge with the type in its low 4 bits}
                                      //     (FP32 evaluations; the FP64 ones read spos and sq_r)
    void* sq_r = nullptr;             // real[N] sorted charges
    int32_t* smol = nullptr;          // [N] sorted molecule ids

    int32_t* core = nullptr;          // [N * cap_core]
    int32_t* ncore = nullptr;         // [N]
    int32_t* shell = nullptr;         // [N * cap_shell] 32-bit sorted indices, or (shell16) 16-bit codes in
                                      //     the first half of the allocation, rows of cap_shell entries
    bool shell16 = false;             // the current shell lists hold 16-bit codes (ListCode)
    int32_t shell_bytes = 4;          // bytes per entry of the shell rows' allocation (2: codes)
    bool shell16_ok = true;           // cleared for good once a build found a row range too long for the codes
    irbe::ListCode lcode{};           // decoding of the current lists' codes
    int32_t* sgroup = nullptr;        // [N] list-build group of each sorted atom (16-bit shell entries)
    int32_t* nshell = nullptr;        // [N]

    void* fsr = nullptr;              // real[3N] sorted short-range (+ excluded-pair) force
    double* pair_part = nullptr;      // [nb * kPairPartials]
    double* fcorr = nullptr;          // [3]
    double* pair_slices = nullptr;    // [256 * 12] first-stage sums of pair_part
    double* ev_pair = nullptr;        // [kPairPartials] reduced pair partials

    int4* kvec = nullptr;             // [P]
    double* kcoef = nullptr;          // [4P]: kx, ky, kz, c_l
    double* rho_part = nullptr;       // [2 * P * nb_rho] (x2 for the adjoint A)
    double* rho = nullptr;            // [2P]
    double* Avec = nullptr;           // [2P]
    void* kforce = nullptr;           // KForce<real>[P]
    void* kadj = nullptr;             // KAdj<real>[P]

    void* gs = nullptr;               // real[3N] sorted dL/dF
    double* gpart = nullptr;          // [nb * 3]
    double* gmean = nullptr;          // [3]
    void* gself = nullptr;            // real[3N]
    void* gscat = nullptr;            // real[3N]
    void* gqself = nullptr;           // real[N]
    void* gqscat = nullptr;           // real[N]
    double* ljpart = nullptr;         // [nb * 2 * kMaxTypesGrad^2]
    double* lj_slices = nullptr;      // [256 * 2 * kMaxTypesGrad^2] first-stage sums of ljpart
    int64_t adj_nb = 0;               // blocks of the last pair-adjoint launch
    int64_t pair_nb = 0;              // blocks of the last pair-force launch
    int64_t part_blocks = 0;          // capacity (blocks) of pair_part and ljpart
    unsigned long long* bk_cursor = nullptr;  // [2 n_c^2] records reserved per destination row, then max |record|
    void* bk_c = nullptr;             // real[4 * bk_total] shell-adjoint records: dL/dr_j (3), dL/dq_j
    uint16_t* bk_j = nullptr;         // [bk_total] record's atom, relative to its row's first atom
    int64_t bk_total = 0;             // allocated records
    unsigned long long* adj_atomics = nullptr;  // [1] shell-adjoint records of the last backward added by atomics
    bool adj_all_atomic = false;      // the last backward added every shell-adjoint record by atomics
    uint16_t* ranks = nullptr;        // [N * p_stride] shell batch ranks of the current step
    int32_t* batch_j = nullptr;       // [N * p_stride] the drawn atoms (sorted index) of the current ranks (with
                                      // stencil sampling -1: i or i's molecule), for the adjoint and read-back:
                                      // written by the forward for the backward that follows it, or decoded
                                      // (stencil ranks, 16-bit shell entries); allocated on first use
    bool batch_j_valid = false;       // batch_j holds the decode of the current ranks
    bool batch_j_fwd = false;         // ... written by a forward (not by a decode for the backward)
    bool keep_batch = false;          // the next forward writes batch_j (the last forward had a backward)
    bool fwd_pending = false;         // a forward ran and no backward has followed it yet
    bool adj_used_batch = false;      // the last backward read batch_j instead of the ranks and shell rows
    int32_t* scell = nullptr;         // [N] stencil sampling: cell of each sorted atom at the last build
    uint32_t* draw_bits = nullptr;    // Floyd bitmaps in device memory for lists too long for LDS
    size_t draw_bits_words = 0;
    int32_t p_stride = 0;
    bool ranks_valid = false;         // ranks hold the draw of ranks_step for the current lists
    uint64_t ranks_step = 0;

    // per-stage event timing (irbe_enable_timing)
    bool timing = false;
    struct Pending {
        int stage;
        hipEvent_t start, stop;
    };
    std::vector<Pending> pending;
    hipEvent_t open_start = nullptr;
    double stage_ms[IRBE_N_STAGES] = {};
    int64_t stage_n[IRBE_N_STAGES] = {};

    std::vector<void*> owned;
};

namespace irbe {

int64_t blocks_for(int64_t n, int block);
int64_t rho_blocks(int64_t n);

// Launchers (all on the handle's stream). Each returns the HIP status of the launch.
hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int32_t v, int64_t n);
hipError_t launch_fill_bytes0(hipStream_t s, void* p, size_t bytes);
hipError_t launch_bin(irbe_ctx* h, const void* pos);
hipError_t launch_requantize(irbe_ctx* h, const void* pos);
hipError_t launch_build_lists(irbe_ctx* h);
hipError_t launch_ksample(irbe_ctx* h, uint64_t step);
hipError_t launch_rho(irbe_ctx* h, const void* grad, bool with_adjoint);
hipError_t launch_pair_forces(irbe_ctx* h, uint64_t step, bool ev);
// True when the shell batch draw of the current lists keeps its Floyd bitmaps in
// LDS (lists of at most 16,384 entries); false when it needs device memory.
bool draw_bitmaps_in_lds(const irbe_ctx* h);
hipError_t launch_pair_reduce(irbe_ctx* h);
hipError_t launch_kspace_forces(irbe_ctx* h, void* force);
hipError_t launch_energy_finalize(irbe_ctx* h, double* ev);
hipError_t launch_sum_q2(irbe_ctx* h);
hipError_t launch_gather_grad(irbe_ctx* h, const void* grad);
hipError_t launch_pair_adjoint(irbe_ctx* h, uint64_t step, bool want_q, bool want_lj);
// Grow the shell-adjoint record buckets to hold `records` records (and create the row cursors).
hipError_t ensure_buckets(irbe_ctx* h, int64_t records);
// Stencil sampling: allocate the read-back array of the decoded batch, and fill it.
hipError_t ensure_batch_atoms(irbe_ctx* h);
// Whether this handle's shell lists can take 16-bit codes (ListCode): split lists
// built by the tiled kernel over a narrow stencil of at most 64 rows.
bool shell16_possible(const irbe_ctx* h);
// Device-memory Floyd bitmaps of at least `words` 32-bit words.
hipError_t ensure_draw_bits(irbe_ctx* h, size_t words);
hipError_t launch_stencil_decode(irbe_ctx* h);
hipError_t launch_kspace_adjoint(irbe_ctx* h, const void* grad, void* grad_pos, void* grad_q, double* grad_lj);

}  // namespace irbe
