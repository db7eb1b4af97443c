/*
 * irbe.h -- C ABI of the MI355X (gfx950) implementation of the non-bonded force
 * of the improved random batch Ewald (IRBE) method:
 *
 *   Liang, Xu, Zhao, "Improved random batch Ewald method in molecular dynamics
 *   simulations", arXiv:2204.13595.
 *
 * The force on atom i is F_i = F_i^core + F_i^shell,* - F^corr + F_i^excl + F_i^long,*:
 *   - F_i^core: exact sum over the core set C(i) = {j != i : r_ij <= r_core}
 *     (Sec. 2.3; the paper's r_eta), pair force of Eq. (2.10);
 *   - F_i^shell,*: (N_S / p_shell) times the sum over a random batch of p_shell
 *     members of the shell set S(i) = {j : r_core < r_ij <= r_shell} (Eq. (2.11);
 *     the paper's r_c), all members with weight 1 when N_S <= p_shell;
 *   - F^corr: the mean of F^core + F^shell,* over all atoms, subtracted from
 *     every atom (Eq. (2.12));
 *   - F_i^excl: removal of the reciprocal-space interaction erf(beta r)/r of
 *     intramolecular (excluded) pairs, which are absent from C(i) and S(i);
 *   - F_i^long,*: the random batch Ewald estimator of Eq. (2.9) over p_kspace
 *     k-vectors drawn from P_k = exp(-k^2/(4 alpha))/S (Eqs. (2.6)-(2.8)),
 *     alpha = beta^2.
 * With p_shell <= 0 the library computes the full-list variant instead: every
 * pair within r_shell with weight 1 and no F^corr (the paper's "RBE" column,
 * RBE without the random batch list).
 *
 * Conventions.
 *   - Units: nm, e, kJ/mol, kJ/mol/nm (coulomb_k = 138.935458 for these).
 *   - Positions, charges, forces and gradients are DEVICE pointers to arrays in
 *     the caller's atom order: positions/forces/gradients [N][3] row-major.
 *     Their element type is float for IRBE_MIXED_FP32 and double for IRBE_FP64.
 *     Arrays whose name ends in _host are host pointers.
 *   - Positions need not be wrapped into the box. Each is stored as a 32-bit
 *     fixed-point fraction of the box, s = rint(frac(x / L) * 2^32) mod 2^32,
 *     so cells, lists and k-space phases are exact integer arithmetic and the
 *     separation of two atoms is the minimum image (requires r_shell < L/2).
 *   - Randomness is counter-based (Philox4x32-10 keyed by the seed): the shell
 *     batch of atom i is a function of (seed, step, i) only, and the k-vectors
 *     of (seed, step) only. Calls with the same step use the same samples.
 *
 * Ownership and streams. The caller owns every pointer argument and keeps the
 * memory alive until the work queued on the handle's stream has completed. The
 * library owns its scratch (allocated in irbe_create / irbe_set_system, grown in
 * irbe_build_lists, freed in irbe_destroy) and keeps no caller pointer across
 * calls. Every call queues work on the stream given to irbe_create and returns
 * without waiting, except irbe_set_system, the first irbe_build_lists of a
 * handle (one wait, to size the list rows; with stencil sampling every build
 * waits once) and the debug/sync calls. A handle is not thread-safe.
 *
 * Errors. Arguments are checked on the host before anything is queued; a bad
 * argument returns IRBE_EINVAL and leaves the handle as it was. Device-side
 * conditions set an error word that the next waiting call (irbe_sync, a
 * waiting irbe_build_lists) reports and clears: IRBE_ENONFINITE for a
 * non-finite position, IRBE_ECAPACITY when a build's lists outgrew their rows
 * (the rows then hold the first entries only, so forces computed from those
 * lists are incomplete; the rows have been grown and the lists must be built
 * again). A queued build also reads back, without waiting, the list lengths of
 * an earlier build once that has completed, and grows the rows for the next
 * builds when they were too short. No call aborts or throws;
 * irbe_last_error() describes the most recent failure.
 */
#ifndef IRBE_H
#define IRBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IRBE_ABI_VERSION 3

typedef struct irbe_ctx* irbe_handle;

typedef enum {
    IRBE_OK = 0,
    IRBE_EINVAL = -1,       /* invalid argument or state                         */
    IRBE_ENOMEM = -2,       /* device allocation failed                          */
    IRBE_EHIP = -3,         /* a HIP runtime call failed                         */
    IRBE_ECAPACITY = -4,    /* a list would exceed the hard capacity limit      */
    IRBE_ESTATE = -5,       /* call out of order (e.g. forces before lists)      */
    IRBE_EUNSUPPORTED = -6, /* valid but outside what this build supports       */
    IRBE_ENONFINITE = -7,   /* non-finite position seen on the device            */
    IRBE_ECONVERGENCE = -8  /* a constraint iteration did not converge           */
} irbe_status;

enum { IRBE_MIXED_FP32 = 0, IRBE_FP64 = 1 };

/* irbe_config.shell_source */
enum { IRBE_SHELL_LIST = 0, IRBE_SHELL_STENCIL = 1 };

/* irbe_config.shell_entries */
enum { IRBE_ENTRIES_AUTO = 0, IRBE_ENTRIES_32 = 32 };

/* compute_forces flags */
enum { IRBE_ENERGY = 1u, IRBE_VIRIAL = 2u };

typedef struct {
    int32_t abi_version;   /* IRBE_ABI_VERSION                                       */
    int32_t precision;     /* IRBE_MIXED_FP32: pair and k-space arithmetic in FP32,
                              structure factor, momentum correction, energies and
                              virial accumulated in FP64; the pair terms (forward
                              and adjoint) take each charge rounded to 19 mantissa
                              bits (relative change below 2^-20), which lets a pair
                              read position, charge and type in one 16-byte load.
                              IRBE_FP64: all FP64, exact charges.                  */
    int64_t n_atoms;       /* N >= 1                                                 */
    double box_length;     /* L, cubic periodic box                                  */
    double ewald_beta;     /* beta = sqrt(alpha): erfc(beta r) real-space split      */
    double coulomb_k;      /* multiplies every Coulomb term                          */
    double r_core;         /* the paper's r_eta; floor(L / r_core) >= 3              */
    double r_shell;        /* the paper's r_c (erfc and LJ cutoff); r_core < r_shell < L/2 */
    int32_t p_shell;       /* shell batch size p~ (> 0), or <= 0 for the full list   */
    int32_t p_kspace;      /* number of sampled k-vectors p (>= 1)                   */
    int32_t n_types;       /* LJ atom types, 1..16                                   */
    int32_t shell_source;  /* where the shell batch is drawn from (p_shell > 0 only):
                              IRBE_SHELL_LIST: S(i), materialized by build_lists,
                              weight N_S / p~ (Eq. (2.11)); IRBE_SHELL_STENCIL:
                              every atom of the shell stencil's cells, K(i)
                              (Algorithm 1 draws the batch from the stencil's
                              cells; Sec. 2.3 lets the distance filter be
                              skipped), weight |K(i)| / p~,
                              a drawn atom counting only when it is in S(i) at
                              the positions given to compute_forces; build_lists
                              then builds no shell list                           */
    uint64_t seed;         /* Philox key                                             */
    double capacity_hint;  /* expected list entries per atom, 0 = from density       */
    double skin;           /* >= 0: lists kept over several steps (Sec. 2.3 lets the
                              cells be slightly larger than r_core so that the lists
                              need not follow every step). Cells of edge
                              >= r_core + skin, C(i) within r_core + skin, S(i)
                              within (r_core - skin, r_shell + skin], the full list
                              within r_shell + skin; compute_forces and
                              compute_gradients count a core entry only at
                              r <= r_core and a shell entry only at
                              r_core < r <= r_shell (full list: r <= r_shell), at
                              the positions they are given. The result equals that
                              of lists built at those positions while no atom has
                              moved more than skin / 2 since build_lists (the caller
                              tracks that and rebuilds); the shell weight uses the
                              list length. floor(L / (r_core + skin)) >= 3 and
                              r_shell + skin < L/2. 0: the lists of Sec. 2.3 as they
                              are, no membership test at force time.            */
    double lj_cut;         /* >= 0: 0 = the LJ term of every listed pair (r <= r_shell),
                              unshifted; > 0 = the shifted-truncated LJ: only at
                              r < lj_cut sigma_ij, its energy shifted to zero there
                              (2^(1/6) for the soft spheres of the paper's
                              primitive-model electrolytes, Sec. 4)              */
    int32_t shell_entries; /* storage of the shell lists S(i) (split lists only):
                              IRBE_ENTRIES_AUTO: 16-bit codes, the member's
                              stencil row and its position in that row's
                              candidate range, where the build of dense cells
                              (>= 4 atoms per cell on average) runs, the shell
                              stencil has at most 64 rows and every row's
                              candidate range fits the code (otherwise, and once
                              a build finds a range too long, 32-bit indices);
                              IRBE_ENTRIES_32: 32-bit sorted indices always.
                              Lists, batches and results are the same either way:
                              the codes halve the shell rows' device memory (2
                              bytes per entry of capacity) and the bytes the list
                              build writes and the pair kernel reads.            */
} irbe_config;

/* Create a handle for one system size and parameter set; work is queued on
 * hip_stream (a hipStream_t; NULL = the default stream). On success *out is a
 * new handle. Returns IRBE_EINVAL for a bad configuration, IRBE_EUNSUPPORTED for
 * one beyond this build's limits (more than 1000 cells per axis, shell stencils
 * wider than 191 cells per axis, stencil sampling over more than 128 stencil
 * rows, k tables too large); the message is in irbe_last_error(NULL). */
irbe_status irbe_create(const irbe_config* cfg, void* hip_stream, irbe_handle* out);

/* Set the topology and parameters (Sec. 2.1: charges q_i, LJ sigma_ij and
 * epsilon_ij per type pair).
 *   type[N] (device, int32 in [0, n_types)), charge[N] (device, float|double),
 *   molecule[N] (device, int32; atoms with the same id >= 0 form excluded pairs,
 *   -1 = no exclusions), lj_sigma_host / lj_eps_host [n_types * n_types] (host,
 *   double, entry [t_i * n_types + t_j] used for the pair (i, j)).
 * Waits on the stream (the exclusion table is built on the host). */
irbe_status irbe_set_system(irbe_handle h, const int32_t* type, const void* charge, const int32_t* molecule,
                            const double* lj_sigma_host, const double* lj_eps_host);

/* Replace charges (device, N) and the LJ tables (host, n_types^2) without
 * touching the topology; NULL leaves that part unchanged. Waits only when LJ
 * tables are given. */
irbe_status irbe_update_parameters(irbe_handle h, const void* charge, const double* lj_sigma_host,
                                   const double* lj_eps_host);

/* Bin atoms into cells and build the core and shell lists (Sec. 2.3;
 * Algorithm 1 builds the core lists of every step) from pos [N][3] (device).
 * Lists are kept until the next call. The first call of a handle (and every
 * call with stencil sampling) waits once to read the list lengths, grows the
 * list rows and builds again when they are too short; later calls queue the
 * build without waiting (see Errors above for rows that turn out too short). */
irbe_status irbe_build_lists(irbe_handle h, const void* pos, uint64_t step);

/* Forces of the last built lists at positions pos (Algorithm 1, force steps):
 * F written to force [N][3] (device, caller order). List membership, N_S and
 * the batch are those of the last build; distances are exact at pos. The
 * samples of `step` are used. With flags & (IRBE_ENERGY | IRBE_VIRIAL),
 * energy_virial (device, 11 doubles) receives
 *   [0] U_coul,short* [1] U_lj* [2] U_long* [3] U_self [4] U_excl
 *   [5..10] W_xx W_yy W_zz W_xy W_xz W_yz,
 * W_ab = sum over pairs of (r_i - r_j)_a f_ij,b plus the k-space term; the
 * starred terms are the estimators matching Eq. (2.3) in expectation.
 * When the last forward of the handle was followed by a backward, a forward with
 * sampled batches also writes its batch atoms (N x p_shell int32 in a buffer that
 * backward allocated; with stencil sampling -1 for the atom itself and its
 * molecule), which irbe_compute_forces_backward at the same step reads in place of
 * the ranks and shell rows, or of decoding the stencil ranks (results bitwise the
 * same); a forward not followed by a backward stops this for the next one. */
irbe_status irbe_compute_forces(irbe_handle h, const void* pos, uint64_t step, void* force, uint32_t flags,
                                double* energy_virial);

/* irbe_compute_forces for callers that cannot allocate device memory during the
 * call (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels, arguments, results and errors, but the
 * per-call scratch of the evaluation (short-range forces in cell order, the
 * per-block partial sums, the momentum correction, the sampled k-vectors, the
 * structure factor and its partials, and the shell batch ranks) is carved from
 * one static device array of 64 MiB per GPU (held until the process ends)
 * instead of the handle's buffers. The call never allocates or frees memory and
 * records no timing events. It needs roughly 3 N real + 2 N ceil4(p_shell)
 * bytes plus the partials (about 230 bytes per atom at p_shell = 100 in mixed
 * precision, i.e. up to ~290,000 atoms); larger systems return IRBE_ECAPACITY,
 * stencil sampling and shell lists longer than 16,384 entries IRBE_EUNSUPPORTED,
 * all before anything is queued. Every call on one GPU shares that GPU's array:
 * calls whose queued work overlaps (on different streams, or from different
 * threads) race and must be serialized by the caller. The array keeps the last
 * call's contents; nothing in it is read before this call writes it. The
 * handle's own state is left as irbe_compute_forces would leave it except that
 * irbe_get_debug's KVEC, RHO, FCORR and BATCH_* selectors still describe the
 * last irbe_compute_forces, and the next backward redraws the batch. */
irbe_status irbe_compute_forces_noalloc(irbe_handle h, const void* pos, uint64_t step, void* force, uint32_t flags,
                                        double* energy_virial);

/* Vector-Jacobian product of irbe_compute_forces at fixed samples and lists:
 * given grad_force = dL/dF [N][3] (device), writes grad_pos = dL/dr [N][3]
 * (device), grad_charge = dL/dq [N] (device, or NULL) and grad_lj =
 * [dL/dsigma (n_types^2), dL/deps (n_types^2)] (device, 2 n_types^2 doubles,
 * or NULL; needs n_types <= 4).
 * Run-to-run reproducibility: the one-sided shell terms dL/dr_j of the batch
 * pairs are staged per block, bucketed by the cell row of j and summed per row
 * in 64-bit fixed point, an order-independent sum, so the result is bitwise
 * reproducible for given inputs. The exceptions, records added with FP atomics
 * whose order varies: all of them with the full list, or when a block's
 * records do not fit the LDS staging (p_shell above 256 in mixed precision,
 * 128 in FP64); single records when a block's staging area or a row's bucket
 * is full, when j's cell row lies outside the stencil window of the block's
 * rows (positions moved far since the build), or when a cell row holds more
 * than 2,048 atoms. irbe_get_debug(IRBE_DBG_ADJ_ATOMICS) returns the number of
 * such records of the last call (-1: all of them). */
irbe_status irbe_compute_forces_backward(irbe_handle h, const void* pos, uint64_t step, const void* grad_force,
                                         void* grad_pos, void* grad_charge, double* grad_lj);

/* Wait for the handle's queued work and report a deferred device error. */
irbe_status irbe_sync(irbe_handle h);

/* Per-stage timing with HIP events recorded on the handle's stream around each
 * kernel (or small kernel group) of the listed stages. enable != 0 starts
 * recording (and clears the totals), 0 stops. irbe_get_timing waits, then
 * writes for each stage s < capacity/2: ms_host[2s] = total milliseconds,
 * ms_host[2s+1] = number of launches; *written = 2 * IRBE_N_STAGES. */
enum {
    IRBE_STAGE_BIN = 0,        /* quantize, histogram, scan, scatter, in-cell sort, gather */
    IRBE_STAGE_LISTS = 1,      /* core/shell list build kernel                             */
    IRBE_STAGE_QUANTIZE = 2,   /* re-quantize positions for a force evaluation             */
    IRBE_STAGE_KSAMPLE = 3,    /* k-vector draw                                            */
    IRBE_STAGE_RHO = 4,        /* structure factor (partials + final reduction)            */
    IRBE_STAGE_PAIR = 5,       /* pair force kernel                                        */
    IRBE_STAGE_PAIR_REDUCE = 6,/* momentum-correction / energy reduction                   */
    IRBE_STAGE_KSPACE = 7,     /* k-space force + final force assembly                     */
    IRBE_STAGE_ENERGY = 8,     /* energy / virial finalisation                             */
    IRBE_STAGE_GRAD_GATHER = 9,/* dL/dF gather and mean                                    */
    IRBE_STAGE_RHO_ADJ = 10,   /* structure factor and A_l (adjoint)                       */
    IRBE_STAGE_PAIR_ADJ = 11,  /* pair adjoint kernel                                      */
    IRBE_STAGE_KSPACE_ADJ = 12,/* k-space adjoint + gradient assembly                      */
    IRBE_N_STAGES = 13
};
irbe_status irbe_enable_timing(irbe_handle h, int32_t enable);
irbe_status irbe_get_timing(irbe_handle h, double* ms_host, int64_t capacity, int64_t* written);

/* Debug/parity read-back (waits). `what` selects the array; dst_host receives
 * up to `capacity` elements; *written = the number of elements available.
 *   IRBE_DBG_CELL_START  int64 [n_c^3 + 1]  atoms of cell c are cell_atoms[cell_start[c]
 *   IRBE_DBG_CELL_ATOMS  int64 [N]          .. cell_start[c+1]), by (fixed-point x, id)
 *   IRBE_DBG_CORE_OFF    int64 [N + 1]      C(i) of atom i (caller order) at
 *   IRBE_DBG_CORE_IDX    int32 [..]         core_idx[core_off[i] .. core_off[i+1]) (atom ids),
 *                                           in stencil-offset order, then cell order
 *   IRBE_DBG_SHELL_OFF   int64 [N + 1]      S(i) (or the full list), same layout
 *   IRBE_DBG_SHELL_IDX   int32 [..]
 *   IRBE_DBG_BATCH_OFF   int64 [N + 1]      batch ranks into S(i) (K(i) with stencil
 *   IRBE_DBG_BATCH_RANK  int32 [..]         sampling), draw order, for the step of
 *                                           the last compute_forces
 *   IRBE_DBG_BATCH_ATOMS int32 [..]         the atoms at those ranks (atom ids; -1
 *                                           for i itself and i's molecule), per-row
 *                                           read-back only
 *   IRBE_DBG_KVEC        int32 [3 P]        sampled m (k = 2 pi m / L)
 *   IRBE_DBG_RHO         double [2 P]       rho(k) (re, im)
 *   IRBE_DBG_FCORR       double [3]         F^corr
 *   IRBE_DBG_SCALARS     double [4]         S, H, n_c, R
 *   IRBE_DBG_COUNTS      int64 [4]          total core entries, total shell (or
 *                                           full-list) entries, row capacities
 *                                           (core, shell) of the last build
 *   IRBE_DBG_ADJ_ATOMICS int64 [1]          shell-adjoint records of the last
 *                                           compute_forces_backward added with FP
 *                                           atomics (-1: all of them)
 *   IRBE_DBG_ADJ_BATCH   int64 [1]          1 when the last compute_forces_backward
 *                                           read the batch atoms written by the
 *                                           forward, 0 when it read the ranks and
 *                                           the shell rows (with 16-bit shell
 *                                           entries: decoded them first into
 *                                           batch atoms)
 *   IRBE_DBG_SHELL_BITS  int64 [1]          storage of the current shell lists:
 *                                           16 (codes) or 32 (sorted indices) */
enum {
    IRBE_DBG_CELL_START = 1,
    IRBE_DBG_CELL_ATOMS = 2,
    IRBE_DBG_CORE_OFF = 3,
    IRBE_DBG_CORE_IDX = 4,
    IRBE_DBG_SHELL_OFF = 5,
    IRBE_DBG_SHELL_IDX = 6,
    IRBE_DBG_BATCH_OFF = 7,
    IRBE_DBG_BATCH_RANK = 8,
    IRBE_DBG_KVEC = 9,
    IRBE_DBG_RHO = 10,
    IRBE_DBG_FCORR = 11,
    IRBE_DBG_SCALARS = 12,
    IRBE_DBG_COUNTS = 13,
    IRBE_DBG_BATCH_ATOMS = 14,
    IRBE_DBG_ADJ_ATOMICS = 15,
    IRBE_DBG_ADJ_BATCH = 16,
    IRBE_DBG_SHELL_BITS = 17
};
irbe_status irbe_get_debug(irbe_handle h, int32_t what, void* dst_host, int64_t capacity, int64_t* written);

/* The same read-back restricted to the atoms rows_host[0..n_rows) (caller ids,
 * host int64), for the per-atom selectors CORE_*, SHELL_* and BATCH_*: the
 * *_OFF selectors give n_rows + 1 offsets, the *_IDX / BATCH_RANK / BATCH_ATOMS
 * selectors the concatenated rows (BATCH_OFF gives the offsets of both). Meant for spot checks on systems too large to copy whole.
 * Waits. IRBE_EINVAL for an id outside [0, N). */
irbe_status irbe_get_debug_rows(irbe_handle h, int32_t what, const int64_t* rows_host, int64_t n_rows, void* dst_host,
                                int64_t capacity, int64_t* written);

/* Message of the last failure on h (or of the last failed irbe_create when h is
 * NULL). The string stays valid until the next call on h. */
const char* irbe_last_error(irbe_handle h);

/* Wait for the handle's work and free everything it owns. */
irbe_status irbe_destroy(irbe_handle h);

/* Measured ceilings of the current HIP device, for reading the roofline
 * figures beside the published peaks; no handle needed. valu_lane_ops_per_s
 * (if not NULL): the rate of full-rate 32-bit integer VALU operations, from
 * independent 24-bit multiply-add chains in every lane of 32 wavefronts per
 * CU (lane operations per second). copy_bytes_per_s (if not NULL): bytes read
 * plus written per second by a streaming 16-byte copy of 1 GiB. Each is timed
 * with HIP events on hip_stream after one untimed launch; the call allocates
 * and frees its own buffers (up to 2 GiB), waits for the stream, and returns
 * IRBE_ENOMEM or IRBE_EHIP on failure. */
irbe_status irbe_probe_rates(void* hip_stream, double* valu_lane_ops_per_s, double* copy_bytes_per_s);

/* ------------------------------------------------------------------------
 * Langevin dynamics (Algorithm 1's last step, "integrate the equations of
 * motion with a thermostat"): the underdamped Langevin equations of Sec. 3,
 * m dv = (F - gamma m v) dt + sqrt(2 gamma m kT) dW, gamma a rate (1/ps),
 * by the splitting kick - drift - noise - drift in leapfrog form with one force
 * evaluation per step, and rigid bond lengths within groups of at most three
 * atoms (rigid water). One step from constrained positions x, velocities v and
 * forces F(x), with w = 1/m:
 *   v += h w F; constrain v (relative velocity along every constraint vector
 *   r_k = x_q - x_p made zero by multiples of r_k weighted by w);
 *   y = x + h/2 v; v = a v + sqrt((1 - a^2) kT w) xi, a = exp(-gamma h);
 *   y += h/2 v; x' = y moved along the r_k (weighted by w) until every
 *   |x'_q - x'_p| equals its length (Newton's method, relative tolerance 1e-14
 *   on the squared lengths); v += (x' - y) / h.
 * xi: per atom, the Philox4x32-10 block of counter (atom, 2^31, step low,
 * 2 * step high) under the key seed, Box-Muller on the word pairs (w0, w1) and
 * (w2, w3) with u = (w + 1) 2^-32 and angle 2 pi w 2^-32. Positions are not
 * wrapped. All state is FP64 (device), in caller atom order.
 * ------------------------------------------------------------------------ */
typedef struct irbe_dyn_ctx* irbe_dyn_handle;

/* irbe_dyn_config.thermostat */
enum { IRBE_LANGEVIN = 0, IRBE_NOSE_HOOVER = 1 };

typedef struct {
    int32_t abi_version;     /* IRBE_ABI_VERSION                                        */
    int32_t force_precision; /* type of the force read and the position copy written:
                                IRBE_MIXED_FP32 float, IRBE_FP64 double                */
    int64_t n_atoms;         /* N >= 1                                                  */
    int64_t n_groups;        /* constraint groups, 1 <= G <= N                          */
    double dt;               /* h > 0 (ps)                                              */
    double gamma;            /* friction rate >= 0 (1/ps)                               */
    double kT;               /* >= 0 (kJ/mol)                                           */
    uint64_t seed;           /* Philox key of the thermostat noise                      */
    int32_t thermostat;      /* IRBE_LANGEVIN, or IRBE_NOSE_HOOVER (the paper's water runs,
                                Sec. 4): the noise step becomes v = exp(-xi h) v (gamma
                                and seed unused) and after the step
                                xi += h (2 K / (n_dof kT) - 1) / tau^2, K the kinetic
                                energy of the new velocities, n_dof = 3 N - (constraints)
                                - 3, xi = 0 at create                                   */
    int32_t reserved;        /* 0                                                       */
    double tau;              /* Nose-Hoover period (ps), > 0 with IRBE_NOSE_HOOVER      */
} irbe_dyn_config;

/* New integrator on hip_stream (a hipStream_t; NULL = the default stream).
 * IRBE_EINVAL for a bad configuration (message in irbe_dyn_last_error(NULL)). */
irbe_status irbe_dyn_create(const irbe_dyn_config* cfg, void* hip_stream, irbe_dyn_handle* out);

/* Topology (device arrays, copied; waits on the stream):
 *   inv_mass[N] (> 0), groups[G][3] (atom indices, -1 = empty slot; slot 0 used;
 *   every atom in exactly one slot), lengths[G][3] (>= 0: the lengths of the
 *   slot pairs (0,1), (0,2), (1,2); a constraint where both slots are used and
 *   the length is > 0). IRBE_EINVAL if any of this does not hold. */
irbe_status irbe_dyn_set_system(irbe_dyn_handle d, const double* inv_mass, const int32_t* groups,
                                const double* lengths);

/* One step in place: pos[N][3], vel[N][3] (device, FP64), force[N][3] (device,
 * float or double per force_precision) = F(pos); `step` keys the noise.
 * pos_copy[N][3] (device, force precision, or NULL) receives the new positions
 * for the next force evaluation. Does not wait; a non-finite result or a
 * constraint iteration that did not converge is reported by irbe_dyn_check. */
irbe_status irbe_dyn_step(irbe_dyn_handle d, double* pos, double* vel, const void* force, uint64_t step,
                          void* pos_copy);

/* out[0] (device FP64) = sum_i m_i |v_i|^2 / 2 (fixed-order sum). Does not wait. */
irbe_status irbe_dyn_kinetic(irbe_dyn_handle d, const double* vel, double* out);

/* out[0] (device FP64) = (1/m) sum_t |pos[sel[t]] - ref[sel[t]]|^2 over the m
 * selected atoms (unwrapped positions; the mean-squared displacement). Does not wait. */
irbe_status irbe_dyn_msd(irbe_dyn_handle d, const double* pos, const double* ref, const int32_t* sel, int64_t m,
                         double* out);

/* Adds to hist[n_bins] (device uint64) the pairs a < b of the m atoms of sel
 * (sel_b NULL), or every pair of an atom of sel and a different atom of the
 * m_b atoms of sel_b, by minimum-image distance r in a cubic box of edge `box` (FP64 without fused
 * operations: d = x_b - x_a - box rint((x_b - x_a) / box) per axis,
 * r = sqrt(d.d)), bin floor(r / (r_max / n_bins)) clamped to the last, r < r_max
 * only; 1 <= n_bins <= 8192. O(m^2) work: an analysis of small systems (the
 * radial distribution function g(r) follows on the host). Does not wait. */
irbe_status irbe_dyn_rdf(irbe_dyn_handle d, const double* pos, const int32_t* sel, int64_t m, const int32_t* sel_b,
                         int64_t m_b, double box, double r_max, int32_t n_bins, uint64_t* hist);

/* out[0..1] (device FP64) = the Nose-Hoover state {xi, sum over steps of h xi}
 * (both 0 with IRBE_LANGEVIN); the quantity U + K + n_dof kT (tau^2 xi^2 / 2 +
 * sum h xi) is conserved by the Nose-Hoover equations. Does not wait. */
irbe_status irbe_dyn_thermostat_state(irbe_dyn_handle d, double* out);

/* n_dof = 3 N - (constraints) - 3 of the topology set (-1 before set_system or for NULL). */
int64_t irbe_dyn_degrees_of_freedom(irbe_dyn_handle d);

/* Waits on the stream and reports device conditions since the last check:
 * IRBE_EINVAL (an msd or rdf selection held an index outside [0, N): those
 * entries were skipped), IRBE_ENONFINITE (non-finite position or velocity),
 * IRBE_ECONVERGENCE. */
irbe_status irbe_dyn_check(irbe_dyn_handle d);

const char* irbe_dyn_last_error(irbe_dyn_handle d);  /* NULL: the last create failure */
irbe_status irbe_dyn_destroy(irbe_dyn_handle d);

#ifdef __cplusplus
}
#endif

#endif /* IRBE_H */
