/*
 * irbe_oracle.c -- plain FP64 CPU oracle for the non-bonded force of the
 * improved random batch Ewald (IRBE) method: the random batch list (RBL) short
 * range combined with the random batch Ewald (RBE) long range.
 *
 * Liang, Xu, Zhao, "Improved random batch Ewald method in molecular dynamics
 * simulations", arXiv:2204.13595.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may load or call this
 * library: only the test suite, the smoke check and the benchmark's CPU
 * baseline leg use it. It shares no source with the HIP implementation; every
 * step is written here from the paper (and from the published definitions of
 * Philox4x32-10, Floyd's sampling algorithm and Lemire's bounded integers).
 *
 * Conventions (readings of the paper where it is silent):
 *  - Positions are represented as 32-bit fixed-point fractions of the box,
 *    s = rint(frac(x / L) * 2^32) mod 2^32. Every distance, cell index and
 *    phase is then exact integer arithmetic; a separation is
 *    d = (int32)(s_j - s_i), whose two's-complement wrap is the minimum image,
 *    and r_ij = r_j - r_i = d * L / 2^32 (Sec. 2.1 defines r_ij = r_j - r_i).
 *  - r_core is the paper's r_eta, r_shell the paper's r_c, beta = sqrt(alpha).
 *  - Every Coulomb term carries the factor ke (Gaussian units when ke = 1).
 *
 * Everything is FP64 and straightforward: no blocking, no fusion, no reordering
 * beyond what the definitions state. OpenMP only splits independent per-atom or
 * per-k work.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TWO32 4294967296.0
#define ORC_TWO64 18446744073709551616.0
#define ORC_PI 3.14159265358979323846

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ECAPACITY = -4, ORC_ENONFINITE = -7 };
enum { ORC_LISTS_SPLIT = 0, ORC_LISTS_FULL = 1, ORC_LISTS_STENCIL = 2 };

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */

/* Fixed-point fractional coordinates of every atom. */
int orc_quantize(int64_t n, double L, const double* pos, uint32_t* s)
{
    const double inv_l = 1.0 / L;
    for (int64_t i = 0; i < 3 * n; ++i) {
        double x = pos[i];
        if (!isfinite(x)) return ORC_ENONFINITE;
        double u = x * inv_l;
        double f = u - floor(u);
        double t = rint(f * ORC_TWO32);
        uint64_t v = (uint64_t)t;
        s[i] = (uint32_t)(v & 0xffffffffu);
    }
    return ORC_OK;
}

/* Number of cells per axis: cells of edge at least r_core (Sec. 2.3, cells of
 * edge r_eta); the 27 nearest cells then hold every core neighbour. */
int32_t orc_n_cells(double L, double r_core) { return (int32_t)floor(L / r_core); }

/* Cells per axis that the shell stencil reaches on each side. */
int32_t orc_shell_reach(double L, double r_shell, int32_t n_c)
{
    return (int32_t)floor(r_shell * (double)n_c / L) + 1;
}

/* Squared radius threshold in quanta^2: D^2 <= T  <=>  r <= radius. */
uint64_t orc_threshold(double radius, double L)
{
    double t = radius * ORC_TWO32 / L;
    return (uint64_t)floor(t * t);
}

static inline int32_t orc_cell_coord(uint32_t s, int32_t n_c)
{
    return (int32_t)(((uint64_t)s * (uint64_t)n_c) >> 32);
}

/* Cell id of atom i: (cz * n_c + cy) * n_c + cx. */
void orc_cell_ids(int64_t n, int32_t n_c, const uint32_t* s, int64_t* cell)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx = orc_cell_coord(s[3 * i + 0], n_c);
        int64_t cy = orc_cell_coord(s[3 * i + 1], n_c);
        int64_t cz = orc_cell_coord(s[3 * i + 2], n_c);
        cell[i] = (cz * n_c + cy) * n_c + cx;
    }
}

/* Per-cell atom lists: cell_start[n_c^3 + 1], cell_atoms[n], ordered by cell
 * id and, inside a cell, by (fixed-point x coordinate, atom id). A counting
 * sort by cell, then an insertion sort of each cell by (s_x, id). */
int orc_cell_lists(int64_t n, int32_t n_c, const uint32_t* s, int64_t* cell_start, int64_t* cell_atoms)
{
    int64_t n_cells = (int64_t)n_c * n_c * n_c;
    int64_t* cell = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* cursor = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_cells);
    if (!cell || !cursor) { free(cell); free(cursor); return ORC_ENOMEM; }
    orc_cell_ids(n, n_c, s, cell);
    memset(cell_start, 0, sizeof(int64_t) * (size_t)(n_cells + 1));
    for (int64_t i = 0; i < n; ++i) cell_start[cell[i] + 1] += 1;
    for (int64_t c = 0; c < n_cells; ++c) cell_start[c + 1] += cell_start[c];
    for (int64_t c = 0; c < n_cells; ++c) cursor[c] = cell_start[c];
    for (int64_t i = 0; i < n; ++i) cell_atoms[cursor[cell[i]]++] = i;
    for (int64_t c = 0; c < n_cells; ++c)
        for (int64_t k = cell_start[c] + 1; k < cell_start[c + 1]; ++k) {
            int64_t v = cell_atoms[k], t = k - 1;
            while (t >= cell_start[c] && (s[3 * cell_atoms[t]] > s[3 * v] ||
                                          (s[3 * cell_atoms[t]] == s[3 * v] && cell_atoms[t] > v))) {
                cell_atoms[t + 1] = cell_atoms[t];
                --t;
            }
            cell_atoms[t + 1] = v;
        }
    free(cell);
    free(cursor);
    return ORC_OK;
}

static inline uint64_t orc_dist2(const uint32_t* s, int64_t i, int64_t j)
{
    uint64_t d2 = 0;
    for (int a = 0; a < 3; ++a) {
        int32_t d = (int32_t)(s[3 * j + a] - s[3 * i + a]);
        d2 += (uint64_t)((int64_t)d * (int64_t)d);
    }
    return d2;
}

static inline int orc_excluded(const int32_t* mol, int64_t i, int64_t j)
{
    return mol != NULL && mol[i] >= 0 && mol[i] == mol[j];
}

/*
 * Core set C(i) = {j != i : r_ij <= r_core} and shell set
 * S(i) = {j : r_core < r_ij <= r_shell} (Sec. 2.3), intramolecular pairs
 * removed. Canonical order: cell offsets (dz, dy, dx) in lexicographic order,
 * then the atoms of each cell in their cell order (by x coordinate, then id). Core offsets are -1..1 on each axis;
 * shell offsets are -R..R when 2R+1 <= n_c, else -h..n_c-1-h with
 * h = floor((n_c-1)/2) (each cell once, and the 27 core cells keep their
 * relative order).
 *
 * Rows are the atoms sel[0..n_sel) (all atoms, in id order, when sel is NULL).
 * Pass 1 (idx == NULL) writes the row counts into *_off[k+1]; pass 2 fills.
 * kind = ORC_LISTS_FULL merges the two sets into one list (core then shell
 * members in a single traversal of the shell stencil), written to the shell
 * arrays. kind = ORC_LISTS_STENCIL writes, in place of S(i), the stencil
 * candidates K(i): every atom of the shell stencil's cells (i itself and its
 * molecule included), in the same canonical order; the random batch is then
 * drawn from K(i) directly (Algorithm 1 draws from the stencil; Sec. 2.3 notes
 * that the filter step can be skipped) and a drawn atom counts only when it
 * is a member of S(i).
 *
 * skin > 0 (lists kept over several steps, Sec. 2.3: cells slightly larger
 * than r_core): the cells have edge >= r_core + skin, C(i) takes
 * r <= r_core + skin, S(i) takes r_core - skin < r <= r_shell + skin (the two
 * overlap), and the full list r <= r_shell + skin; a force evaluation then
 * counts an entry only when the pair is a member at its own positions. skin = 0
 * gives the sets above exactly.
 */
static int64_t orc_list_row(int64_t i, const uint32_t* s, const int32_t* mol, int32_t n_c, int32_t R,
                            uint64_t t_core, uint64_t t_lo, uint64_t t_shell, const int64_t* cell_start,
                            const int64_t* cell_atoms, int want_core, int full_list, int32_t* out)
{
    int64_t count = 0;
    int32_t cx = orc_cell_coord(s[3 * i + 0], n_c);
    int32_t cy = orc_cell_coord(s[3 * i + 1], n_c);
    int32_t cz = orc_cell_coord(s[3 * i + 2], n_c);
    int32_t lo, hi;
    if (want_core) {
        lo = -1; hi = 1;
    } else if (2 * R + 1 <= n_c) {
        lo = -R; hi = R;
    } else {
        lo = -((n_c - 1) / 2); hi = lo + n_c - 1;
    }
    for (int32_t dz = lo; dz <= hi; ++dz)
        for (int32_t dy = lo; dy <= hi; ++dy)
            for (int32_t dx = lo; dx <= hi; ++dx) {
                int64_t x = ((cx + dx) % n_c + n_c) % n_c;
                int64_t y = ((cy + dy) % n_c + n_c) % n_c;
                int64_t z = ((cz + dz) % n_c + n_c) % n_c;
                int64_t c = (z * n_c + y) * n_c + x;
                for (int64_t k = cell_start[c]; k < cell_start[c + 1]; ++k) {
                    int64_t j = cell_atoms[k];
                    int take;
                    if (!want_core && full_list == ORC_LISTS_STENCIL) {
                        take = 1;
                    } else {
                        if (j == i || orc_excluded(mol, i, j)) continue;
                        uint64_t d2 = orc_dist2(s, i, j);
                        if (want_core) take = d2 <= t_core;
                        else if (full_list == ORC_LISTS_FULL) take = d2 <= t_shell;
                        else take = d2 > t_lo && d2 <= t_shell;
                    }
                    if (take) {
                        if (out) out[count] = (int32_t)j;
                        ++count;
                    }
                }
            }
    return count;
}

int orc_build_lists(int64_t n, const uint32_t* s, const int32_t* mol, double L, double r_core,
                    double r_shell, double skin, int full_list, const int64_t* sel, int64_t n_sel,
                    int64_t* core_off, int32_t* core_idx, int64_t* shell_off, int32_t* shell_idx)
{
    if (!(skin >= 0.0)) return ORC_EINVAL;
    int32_t n_c = orc_n_cells(L, r_core + skin);
    if (n_c < 3 || !(r_shell > r_core) || !(r_shell + skin < 0.5 * L)) return ORC_EINVAL;
    int32_t R = orc_shell_reach(L, r_shell + skin, n_c);
    uint64_t t_core = orc_threshold(r_core + skin, L);
    uint64_t t_lo = r_core > skin ? orc_threshold(r_core - skin, L) : 0;
    uint64_t t_shell = orc_threshold(r_shell + skin, L);
    int64_t n_cells = (int64_t)n_c * n_c * n_c;
    int64_t* cell_start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_cells + 1));
    int64_t* cell_atoms = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!cell_start || !cell_atoms) { free(cell_start); free(cell_atoms); return ORC_ENOMEM; }
    orc_cell_lists(n, n_c, s, cell_start, cell_atoms);
    int64_t rows = sel ? n_sel : n;
    int fill = core_idx != NULL || shell_idx != NULL;
    if (!fill) {
        core_off[0] = 0;
        shell_off[0] = 0;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < rows; ++k) {
        int64_t i = sel ? sel[k] : k;
        if (!fill) {
            core_off[k + 1] = full_list == ORC_LISTS_FULL
                                  ? 0
                                  : orc_list_row(i, s, mol, n_c, R, t_core, t_lo, t_shell, cell_start, cell_atoms, 1, 0, NULL);
            shell_off[k + 1] = orc_list_row(i, s, mol, n_c, R, t_core, t_lo, t_shell, cell_start, cell_atoms, 0,
                                            full_list, NULL);
        } else {
            if (full_list != ORC_LISTS_FULL && core_idx)
                orc_list_row(i, s, mol, n_c, R, t_core, t_lo, t_shell, cell_start, cell_atoms, 1, 0, core_idx + core_off[k]);
            if (shell_idx)
                orc_list_row(i, s, mol, n_c, R, t_core, t_lo, t_shell, cell_start, cell_atoms, 0, full_list,
                             shell_idx + shell_off[k]);
        }
    }
    if (!fill)
        for (int64_t k = 0; k < rows; ++k) {
            core_off[k + 1] += core_off[k];
            shell_off[k + 1] += shell_off[k];
        }
    free(cell_start);
    free(cell_atoms);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,  */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).                    */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A stream of 32-bit words: block b is Philox(counter = {c0, b, c2, c3},
 * key = {seed lo, seed hi}), read word 0..3 in turn.
 * c2 = low 32 bits of the step; c3 = (high 32 bits of the step) * 2 + tag,
 * tag 0 for the shell batch (c0 = atom id), 1 for the k draw (c0 = sample). */
typedef struct {
    uint32_t key[2];
    uint32_t c0, c2, c3;
    uint32_t block;
    uint32_t buf[4];
    int pos;
} orc_stream;

static void orc_stream_init(orc_stream* st, uint64_t seed, uint64_t step, uint32_t c0, uint32_t tag)
{
    st->key[0] = (uint32_t)seed;
    st->key[1] = (uint32_t)(seed >> 32);
    st->c0 = c0;
    st->c2 = (uint32_t)step;
    st->c3 = ((uint32_t)(step >> 32) << 1) | (tag & 1u);
    st->block = 0;
    st->pos = 4;
}

static uint32_t orc_stream_next(orc_stream* st)
{
    if (st->pos == 4) {
        uint32_t ctr[4] = {st->c0, st->block, st->c2, st->c3};
        orc_philox4x32_10(ctr, st->key, st->buf);
        st->block += 1;
        st->pos = 0;
    }
    return st->buf[st->pos++];
}

/* Words of the Langevin thermostat noise: for atom c0 = 0 .. n-1 the four
 * words of the Philox block with counter (c0, 2^31, step low, 2 * step high)
 * under the key seed. The shell batch streams use blocks below 2^31 (a row
 * would need 2^33 draws to reach it) and the k draw has tag 1 in c3, so the
 * three never share a counter. */
void orc_noise_words(uint64_t seed, uint64_t step, int64_t n, uint32_t* out)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < n; ++i) {
        uint32_t ctr[4] = {(uint32_t)i, 0x80000000u, (uint32_t)step, (uint32_t)(step >> 32) << 1};
        orc_philox4x32_10(ctr, key, out + 4 * i);
    }
}

/* Uniform integer in [0, n), n >= 1: Lemire's multiply-shift with rejection
 * ("Fast random integer generation in an interval", 2019). */
static uint32_t orc_uniform_below(orc_stream* st, uint32_t n)
{
    uint64_t m = (uint64_t)orc_stream_next(st) * (uint64_t)n;
    uint32_t l = (uint32_t)m;
    if (l < n) {
        uint32_t thr = (uint32_t)(0u - n) % n;
        while (l < thr) {
            m = (uint64_t)orc_stream_next(st) * (uint64_t)n;
            l = (uint32_t)m;
        }
    }
    return (uint32_t)(m >> 32);
}

/*
 * Shell batch of atom `id` (Sec. 2.3, Eq. (2.11); Algorithm 1 picks p~ of the
 * shell particles, or all of them when N_S <= p~). Sampling is without
 * replacement (Floyd's algorithm): for t = N_S - p .. N_S - 1 draw r uniform
 * in [0, t]; insert r, or t when r is already in the batch. Ranks index S(i)
 * in its canonical order and are written in insertion order. Returns the batch
 * size.
 */
int32_t orc_shell_ranks(uint64_t seed, uint64_t step, int64_t id, int32_t n_s, int32_t p_s, int32_t* ranks)
{
    if (n_s <= p_s) {
        for (int32_t r = 0; r < n_s; ++r) ranks[r] = r;
        return n_s;
    }
    orc_stream st;
    orc_stream_init(&st, seed, step, (uint32_t)id, 0u);
    unsigned char* taken = (unsigned char*)calloc((size_t)n_s, 1);
    int32_t count = 0;
    for (int32_t t = n_s - p_s; t < n_s; ++t) {
        int32_t r = (int32_t)orc_uniform_below(&st, (uint32_t)t + 1u);
        int32_t pick = taken[r] ? t : r;
        taken[pick] = 1;
        ranks[count++] = pick;
    }
    free(taken);
    return count;
}

/* ------------------------------------------------------------------------ */
/* Importance sampling of k (Sec. 2.2, Eqs. (2.6)-(2.8)).                    */
/* ------------------------------------------------------------------------ */

/* Per-axis weight of k = 2 pi m / L: exp(-k^2/(4 alpha)) = exp(-(pi m/(beta L))^2). */
static double orc_axis_weight(double a, int32_t m)
{
    double x = a * (double)m;
    return exp(-(x * x));
}

/*
 * Per-axis table of the discrete Gaussian. M is the smallest m >= 0 whose
 * successor weight is below 2^-64. H = sum_{m=-M..M} w(m) (Eq. (2.7), left
 * form, summed in ascending m) and S = H^3 - 1 (Eq. (2.6)). U[m + M] =
 * floor(2^64 * cdf(m)) with cdf accumulated in ascending m; U[2M] = 2^64 - 1.
 * Returns M, or -1 when M would exceed max_m.
 */
int32_t orc_ktable(double beta, double L, int32_t max_m, uint64_t* U, double* H_out, double* S_out)
{
    double a = ORC_PI / (beta * L);
    int32_t M = 0;
    while (orc_axis_weight(a, M + 1) >= 1.0 / ORC_TWO64) {
        ++M;
        if (M > max_m) return -1;
    }
    double H = 0.0;
    for (int32_t m = -M; m <= M; ++m) H += orc_axis_weight(a, m);
    if (U) {
        double c = 0.0;
        for (int32_t m = -M; m <= M; ++m) {
            c += orc_axis_weight(a, m);
            double x = (c / H) * ORC_TWO64;
            U[m + M] = (x >= ORC_TWO64) ? UINT64_MAX : (uint64_t)x;
        }
        U[2 * M] = UINT64_MAX;
    }
    if (H_out) *H_out = H;
    if (S_out) *S_out = H * H * H - 1.0;
    return M;
}

/* P k-vectors m_l (k_l = 2 pi m_l / L) drawn i.i.d. from P_k (Eq. (2.8)):
 * per axis, a 64-bit word u (first 32-bit word high) picks the least m with
 * u < U[m + M]; a triple (0,0,0) is drawn again from the next words. */
void orc_kdraw(uint64_t seed, uint64_t step, int32_t P, int32_t M, const uint64_t* U, int32_t* m_out)
{
    for (int32_t l = 0; l < P; ++l) {
        orc_stream st;
        orc_stream_init(&st, seed, step, (uint32_t)l, 1u);
        int32_t m[3];
        do {
            for (int a = 0; a < 3; ++a) {
                uint64_t hi = orc_stream_next(&st);
                uint64_t lo = orc_stream_next(&st);
                uint64_t u = (hi << 32) | lo;
                int32_t v = M;
                for (int32_t t = -M; t < M; ++t)
                    if (u < U[t + M]) { v = t; break; }
                m[a] = v;
            }
        } while (m[0] == 0 && m[1] == 0 && m[2] == 0);
        m_out[3 * l + 0] = m[0];
        m_out[3 * l + 1] = m[1];
        m_out[3 * l + 2] = m[2];
    }
}

/* ------------------------------------------------------------------------ */
/* Forces and energies                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    double L;        /* box edge (nm) */
    double beta;     /* Ewald splitting: the paper's alpha is beta^2 */
    double ke;       /* Coulomb constant */
    int32_t n_types; /* LJ tables are n_types x n_types, entry [t_i * n_types + t_j] */
    double lj_cut;   /* > 0: LJ only at r < lj_cut sigma_ij, shifted by -u_LJ(lj_cut sigma_ij) (the
                        shifted-truncated LJ of the primitive-model electrolytes, Sec. 4, with
                        lj_cut = 2^(1/6)); 0: LJ over every listed pair, unshifted */
} orc_system;

/* Whether the LJ term acts at distance r (pair parameters sig). */
static inline int orc_lj_on(const orc_system* sy, double sig, double r)
{
    return sy->lj_cut <= 0.0 || r < sy->lj_cut * sig;
}

/* Pair force f_ij = phi(r) r_ij of Eq. (2.10) (erfc + Gaussian Coulomb, LJ),
 * and the pair energy u_ij = ke q_i q_j erfc(beta r)/r + 4 eps((s/r)^12-(s/r)^6)
 * split as (Coulomb, LJ) (Eq. (2.3)). */
static void orc_pair(const orc_system* sy, double qi, double qj, double sig, double eps, double r,
                     double* phi, double* u_coul, double* u_lj)
{
    const double b = sy->beta;
    double erfc_br = erfc(b * r);
    double gauss = 2.0 * b / sqrt(ORC_PI) * exp(-b * b * r * r);
    double coul = -sy->ke * qi * qj * (erfc_br / (r * r) + gauss / r) / r;
    double lj = 0.0, ulj = 0.0;
    if (eps != 0.0 && orc_lj_on(sy, sig, r)) {
        double s6 = pow(sig, 6), s12 = s6 * s6;
        lj = -eps * (48.0 * s12 / pow(r, 14) - 24.0 * s6 / pow(r, 8));
        ulj = 4.0 * eps * (s12 / pow(r, 12) - s6 / pow(r, 6));
        if (sy->lj_cut > 0.0) {
            double k6 = pow(sy->lj_cut, -6);
            ulj -= 4.0 * eps * (k6 * k6 - k6);
        }
    }
    *phi = coul + lj;
    *u_coul = sy->ke * qi * qj * erfc_br / r;
    *u_lj = ulj;
}

static inline void orc_sep(const uint32_t* s, int64_t i, int64_t j, double L, double dv[3], double* r)
{
    const double q = L / ORC_TWO32;
    double r2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        dv[a] = (double)(int32_t)(s[3 * j + a] - s[3 * i + a]) * q;
        r2 += dv[a] * dv[a];
    }
    *r = sqrt(r2);
}


/* Row r of a step: atom rows[r], or atom r when rows is NULL. */
static inline int64_t orc_row_atom(const int64_t* rows, int64_t r) { return rows ? rows[r] : r; }

/*
 * Short-range force of Eqs. (2.10)-(2.11), before the momentum correction:
 *   F_i = sum_{j in C(i)} f_ij + w_i sum_{j in B(i)} f_ij
 * for each row atom i. core_off/core_idx hold C(i) per row (may be NULL: empty);
 * shell_off/shell_idx hold S(i) per row; the batch B(i) is given as ranks into
 * S(i) (batch_off/batch_rank per row; NULL: every member); w per row (NULL: 1).
 * core_accept / accept (NULL: all) flag the core and batch entries that count
 * (stencil sampling, skin lists).
 * e8 accumulates [U_coul, U_lj, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz] with the
 * estimator U = 1/2 sum_i (sum_C u_ij + w_i sum_B u_ij), and likewise for the
 * pair virial W_ab = -1/2 sum_i sum_j w r_ij,a f_ij,b.
 */
int orc_short_range(const orc_system* sy, int64_t n, const uint32_t* s, const double* q, const int32_t* type,
                    const double* lj_sigma, const double* lj_eps, const int64_t* rows, int64_t n_rows,
                    const int64_t* core_off, const int32_t* core_idx, const int64_t* shell_off,
                    const int32_t* shell_idx, const int64_t* batch_off, const int32_t* batch_rank,
                    const double* w, const uint8_t* core_accept, const uint8_t* accept, double* f_out, double* e8)
{
    (void)n;
    const int nt = sy->n_types;
    double tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma omp parallel
    {
        double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n_rows; ++r) {
            int64_t i = orc_row_atom(rows, r);
            double wi = w ? w[r] : 1.0;
            double f[3] = {0, 0, 0};
            for (int pass = 0; pass < 2; ++pass) {
                int64_t cnt;
                if (pass == 0) cnt = core_off ? core_off[r + 1] - core_off[r] : 0;
                else cnt = batch_off ? batch_off[r + 1] - batch_off[r] : shell_off[r + 1] - shell_off[r];
                double scale = pass == 0 ? 1.0 : wi;
                for (int64_t k = 0; k < cnt; ++k) {
                    int64_t j;
                    if (pass == 0) j = core_idx[core_off[r] + k];
                    else j = shell_idx[shell_off[r] + (batch_off ? batch_rank[batch_off[r] + k] : k)];
                    if (pass == 0 && core_accept && !core_accept[core_off[r] + k]) continue;
                    if (pass == 1 && accept && !accept[(batch_off ? batch_off[r] : shell_off[r]) + k]) continue;
                    double dv[3], dist, phi, uc, ul;
                    orc_sep(s, i, j, sy->L, dv, &dist);
                    int tp = type[i] * nt + type[j];
                    orc_pair(sy, q[i], q[j], lj_sigma[tp], lj_eps[tp], dist, &phi, &uc, &ul);
                    for (int a = 0; a < 3; ++a) f[a] += scale * phi * dv[a];
                    part[0] += 0.5 * scale * uc;
                    part[1] += 0.5 * scale * ul;
                    part[2] += -0.5 * scale * dv[0] * phi * dv[0];
                    part[3] += -0.5 * scale * dv[1] * phi * dv[1];
                    part[4] += -0.5 * scale * dv[2] * phi * dv[2];
                    part[5] += -0.5 * scale * dv[0] * phi * dv[1];
                    part[6] += -0.5 * scale * dv[0] * phi * dv[2];
                    part[7] += -0.5 * scale * dv[1] * phi * dv[2];
                }
            }
            for (int a = 0; a < 3; ++a) f_out[3 * r + a] = f[a];
        }
#pragma omp critical
        for (int c = 0; c < 8; ++c) tot[c] += part[c];
    }
    if (e8)
        for (int c = 0; c < 8; ++c) e8[c] += tot[c];
    return ORC_OK;
}

/*
 * Excluded (same-molecule) pairs. The reciprocal sum counts every pair, so the
 * excluded pair's erf(beta r)/r interaction is removed (minimum image, no
 * cutoff): U -= ke q_i q_j erf(beta r)/r and the matching force
 *   F_i += psi(r) r_ij,  psi = -ke q_i q_j (2 beta e^{-beta^2 r^2}/(sqrt(pi) r) - erf(beta r)/r^2)/r.
 * excl_off/excl_idx: the partners of each row atom. e7 accumulates
 * [U_excl, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz].
 */
int orc_exclusions(const orc_system* sy, const uint32_t* s, const double* q, const int64_t* rows, int64_t n_rows,
                   const int64_t* excl_off, const int64_t* excl_idx, double* f_out, double* e7)
{
    const double b = sy->beta;
    double tot[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t i = orc_row_atom(rows, r);
        double f[3] = {0, 0, 0};
        for (int64_t k = excl_off[r]; k < excl_off[r + 1]; ++k) {
            int64_t j = excl_idx[k];
            double dv[3], dist;
            orc_sep(s, i, j, sy->L, dv, &dist);
            double e = erf(b * dist);
            double g = 2.0 * b / sqrt(ORC_PI) * exp(-b * b * dist * dist);
            double psi = -sy->ke * q[i] * q[j] * (g / dist - e / (dist * dist)) / dist;
            for (int a = 0; a < 3; ++a) f[a] += psi * dv[a];
            tot[0] += 0.5 * (-sy->ke * q[i] * q[j] * e / dist);
            tot[1] += -0.5 * dv[0] * psi * dv[0];
            tot[2] += -0.5 * dv[1] * psi * dv[1];
            tot[3] += -0.5 * dv[2] * psi * dv[2];
            tot[4] += -0.5 * dv[0] * psi * dv[1];
            tot[5] += -0.5 * dv[0] * psi * dv[2];
            tot[6] += -0.5 * dv[1] * psi * dv[2];
        }
        for (int a = 0; a < 3; ++a) f_out[3 * r + a] = f[a];
    }
    if (e7)
        for (int c = 0; c < 7; ++c) e7[c] += tot[c];
    return ORC_OK;
}

/* Exact phase k_l . r_j = 2 pi ((m_l . s_j) mod 2^32) / 2^32, as an angle in [-pi, pi). */
static inline double orc_phase(const int32_t* m, const uint32_t* sj)
{
    uint32_t ph = (uint32_t)m[0] * sj[0] + (uint32_t)m[1] * sj[1] + (uint32_t)m[2] * sj[2];
    return 2.0 * ORC_PI * (double)(int32_t)ph / ORC_TWO32;
}

/* Structure factor rho(k_l) = sum_j q_j e^{i k_l . r_j} (Eq. (2.4)) over the
 * row atoms (all atoms when rows is NULL): rho_out[2l] = Re, rho_out[2l+1] = Im. */
int orc_structure_factor(const uint32_t* s, const double* q, const int64_t* rows, int64_t n_rows, int32_t n_k,
                         const int32_t* kvec, double* rho_out)
{
#pragma omp parallel for schedule(static)
    for (int32_t l = 0; l < n_k; ++l) {
        double re = 0.0, im = 0.0;
        for (int64_t r = 0; r < n_rows; ++r) {
            int64_t j = orc_row_atom(rows, r);
            double th = orc_phase(kvec + 3 * l, s + 3 * j);
            re += q[j] * cos(th);
            im += q[j] * sin(th);
        }
        rho_out[2 * l + 0] = re;
        rho_out[2 * l + 1] = im;
    }
    return ORC_OK;
}

/*
 * Long-range force on each row atom for the listed k (Eq. (2.9); with
 * W_l = exp(-k^2/(4 alpha)) over all k != 0 it is F^long of Eq. (2.5)):
 *   F_i = -ke q_i sum_l W_l 4 pi k_l / (V |k_l|^2) Im(e^{-i k_l.r_i} rho_l).
 */
int orc_kspace_force(const orc_system* sy, const uint32_t* s, const double* q, const int64_t* rows,
                     int64_t n_rows, int32_t n_k, const int32_t* kvec, const double* wk, const double* rho,
                     double* f_out)
{
    const double L = sy->L, V = L * L * L, tpl = 2.0 * ORC_PI / L;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t i = orc_row_atom(rows, r);
        double f[3] = {0, 0, 0};
        for (int32_t l = 0; l < n_k; ++l) {
            double k[3] = {tpl * kvec[3 * l], tpl * kvec[3 * l + 1], tpl * kvec[3 * l + 2]};
            double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            double th = orc_phase(kvec + 3 * l, s + 3 * i);
            double im = rho[2 * l + 1] * cos(th) - rho[2 * l] * sin(th);
            double c = -sy->ke * q[i] * wk[l] * 4.0 * ORC_PI / (V * k2) * im;
            for (int a = 0; a < 3; ++a) f[a] += c * k[a];
        }
        for (int a = 0; a < 3; ++a) f_out[3 * r + a] = f[a];
    }
    return ORC_OK;
}

/*
 * Long-range energy U = ke sum_l W_l 2 pi |rho_l|^2 / (V |k_l|^2) (Eq. (2.3))
 * and its virial W_ab = sum_l U_l (delta_ab - 2 k_a k_b (1/k^2 + 1/(4 alpha)))
 * (minus the derivative of U under a homogeneous strain of box and positions).
 * e7 accumulates [U_long, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz].
 */
int orc_kspace_energy(const orc_system* sy, int32_t n_k, const int32_t* kvec, const double* wk, const double* rho,
                      double* e7)
{
    const double L = sy->L, V = L * L * L, tpl = 2.0 * ORC_PI / L;
    const double alpha = sy->beta * sy->beta;
    for (int32_t l = 0; l < n_k; ++l) {
        double k[3] = {tpl * kvec[3 * l], tpl * kvec[3 * l + 1], tpl * kvec[3 * l + 2]};
        double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        double rho2 = rho[2 * l] * rho[2 * l] + rho[2 * l + 1] * rho[2 * l + 1];
        double u = sy->ke * wk[l] * 2.0 * ORC_PI * rho2 / (V * k2);
        double g = 2.0 * (1.0 / k2 + 1.0 / (4.0 * alpha));
        e7[0] += u;
        e7[1] += u * (1.0 - g * k[0] * k[0]);
        e7[2] += u * (1.0 - g * k[1] * k[1]);
        e7[3] += u * (1.0 - g * k[2] * k[2]);
        e7[4] += u * (-g * k[0] * k[1]);
        e7[5] += u * (-g * k[0] * k[2]);
        e7[6] += u * (-g * k[1] * k[2]);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Adjoint: gradients of L = sum_i G_i . F_i with the lists, batches and k   */
/* frozen. F_i = F_i^sr - F^corr + F_i^excl + F_i^long.                      */
/* ------------------------------------------------------------------------ */

/*
 * Short-range adjoint, plain scatter form. With f_ij = phi(r) r_ij and the
 * batch weight c (1 for core pairs, w_i for batch pairs), the loss term is
 * c Gs_i . f_ij where Gs = G - mean(G) when the momentum correction is applied
 * (rbl != 0) and Gs = G otherwise. With J = phi I + (phi'(r)/r) r_ij r_ij^T:
 *   dL/dr_j += c J Gs_i,  dL/dr_i -= c J Gs_i,
 *   dL/dq_i += c Gs_i . (d f_ij/d q_i), dL/dq_j += c Gs_i . (d f_ij / d q_j),
 *   dL/dsigma[t_i t_j], dL/deps[t_i t_j] likewise.
 * Runs over every atom (rows are all atoms). Outputs are accumulated.
 */
/* The terms are those of G'_i . F_i for each listed atom i (rows, or all atoms
 * when rows is NULL; the lists are per row): for a dL/dF that vanishes outside
 * the rows and sums to zero, the rows' terms are all the short-range terms. */
int orc_short_range_adjoint(const orc_system* sy, int64_t n, const uint32_t* s, const double* q,
                            const int32_t* type, const double* lj_sigma, const double* lj_eps, const int64_t* rows,
                            int64_t n_rows, const int64_t* core_off, const int32_t* core_idx,
                            const int64_t* shell_off, const int32_t* shell_idx, const int64_t* batch_off,
                            const int32_t* batch_rank, const double* w, const uint8_t* core_accept,
                            const uint8_t* accept, int rbl, const double* G, double* g_pos, double* g_q,
                            double* g_sigma, double* g_eps)
{
    const int nt = sy->n_types;
    const double b = sy->beta, ke = sy->ke, spi = sqrt(ORC_PI);
    double mean[3] = {0, 0, 0};
    if (rbl && n > 0) {
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) mean[a] += G[3 * i + a];
        for (int a = 0; a < 3; ++a) mean[a] /= (double)n;
    }
    for (int64_t r = 0; r < n_rows; ++r) {
        const int64_t i = orc_row_atom(rows, r);
        double gi[3] = {G[3 * i] - mean[0], G[3 * i + 1] - mean[1], G[3 * i + 2] - mean[2]};
        for (int pass = 0; pass < 2; ++pass) {
            int64_t cnt;
            if (pass == 0) cnt = core_off ? core_off[r + 1] - core_off[r] : 0;
            else cnt = batch_off ? batch_off[r + 1] - batch_off[r] : shell_off[r + 1] - shell_off[r];
            double c = pass == 0 ? 1.0 : (w ? w[r] : 1.0);
            for (int64_t k = 0; k < cnt; ++k) {
                int64_t j;
                if (pass == 0) j = core_idx[core_off[r] + k];
                else j = shell_idx[shell_off[r] + (batch_off ? batch_rank[batch_off[r] + k] : k)];
                if (pass == 0 && core_accept && !core_accept[core_off[r] + k]) continue;
                if (pass == 1 && accept && !accept[(batch_off ? batch_off[r] : shell_off[r]) + k]) continue;
                double dv[3], r;
                orc_sep(s, i, j, sy->L, dv, &r);
                int tp = type[i] * nt + type[j];
                double sig = lj_sigma[tp], eps = lj_eps[tp];
                /* Coulomb: phi_c = -ke qi qj (A + B) with A = erfc(br)/r^3, B = 2b e^{-b^2r^2}/(sqrt(pi) r^2) */
                double ex = exp(-b * b * r * r);
                double A = erfc(b * r) / (r * r * r);
                double B = 2.0 * b / spi * ex / (r * r);
                double dA = -2.0 * b / spi * ex / (r * r * r) - 3.0 * erfc(b * r) / (r * r * r * r);
                double dB = -2.0 * b / spi * ex * (2.0 * b * b / r + 2.0 / (r * r * r));
                double phi = -ke * q[i] * q[j] * (A + B);
                double dphi = -ke * q[i] * q[j] * (dA + dB);
                double C = 0.0, dC = 0.0, dC_dsig = 0.0;
                if ((eps != 0.0 || sig != 0.0) && orc_lj_on(sy, sig, r)) {
                    C = 48.0 * pow(sig, 12) / pow(r, 14) - 24.0 * pow(sig, 6) / pow(r, 8);
                    dC = -672.0 * pow(sig, 12) / pow(r, 15) + 192.0 * pow(sig, 6) / pow(r, 9);
                    dC_dsig = 576.0 * pow(sig, 11) / pow(r, 14) - 144.0 * pow(sig, 5) / pow(r, 8);
                }
                phi += -eps * C;
                dphi += -eps * dC;
                double gd = gi[0] * dv[0] + gi[1] * dv[1] + gi[2] * dv[2];
                for (int a = 0; a < 3; ++a) {
                    double jg = phi * gi[a] + dphi / r * dv[a] * gd;
                    g_pos[3 * j + a] += c * jg;
                    g_pos[3 * i + a] -= c * jg;
                }
                if (g_q) {
                    g_q[i] += c * (-ke * q[j] * (A + B)) * gd;
                    g_q[j] += c * (-ke * q[i] * (A + B)) * gd;
                }
                if (g_eps) g_eps[tp] += c * (-C) * gd;
                if (g_sigma) g_sigma[tp] += c * (-eps * dC_dsig) * gd;
            }
        }
    }
    return ORC_OK;
}

/* Adjoint of the excluded-pair correction (uses G itself: the momentum
 * correction does not cover it). excl lists are per atom over all atoms. */
int orc_exclusions_adjoint(const orc_system* sy, const uint32_t* s, const double* q, const int64_t* rows,
                           int64_t n_rows, const int64_t* excl_off, const int64_t* excl_idx, const double* G,
                           double* g_pos, double* g_q)
{
    const double b = sy->beta, ke = sy->ke, spi = sqrt(ORC_PI);
    for (int64_t r = 0; r < n_rows; ++r) {
        const int64_t i = orc_row_atom(rows, r);
        for (int64_t k = excl_off[r]; k < excl_off[r + 1]; ++k) {
            int64_t j = excl_idx[k];
            double dv[3], r;
            orc_sep(s, i, j, sy->L, dv, &r);
            double ex = exp(-b * b * r * r);
            double Bx = 2.0 * b / spi * ex / (r * r);
            double E = erf(b * r) / (r * r * r);
            double dBx = -2.0 * b / spi * ex * (2.0 * b * b / r + 2.0 / (r * r * r));
            double dE = 2.0 * b / spi * ex / (r * r * r) - 3.0 * erf(b * r) / (r * r * r * r);
            double psi = -ke * q[i] * q[j] * (Bx - E);
            double dpsi = -ke * q[i] * q[j] * (dBx - dE);
            const double* gi = G + 3 * i;
            double gd = gi[0] * dv[0] + gi[1] * dv[1] + gi[2] * dv[2];
            for (int a = 0; a < 3; ++a) {
                double jg = psi * gi[a] + dpsi / r * dv[a] * gd;
                g_pos[3 * j + a] += jg;
                g_pos[3 * i + a] -= jg;
            }
            if (g_q) {
                g_q[i] += -ke * q[j] * (Bx - E) * gd;
                g_q[j] += -ke * q[i] * (Bx - E) * gd;
            }
        }
    }
    return ORC_OK;
}

/*
 * Adjoint of the long-range force of Eq. (2.9) for the listed k (weights W_l).
 * With c_l = W_l 4 pi/(V |k_l|^2), g_nl = G_n . k_l, theta_nl = k_l . r_n and
 * A_l = sum_m q_m g_ml e^{i theta_ml}:
 *   dL/dr_n = -ke q_n sum_l c_l k_l [Re(e^{i theta_nl} conj(A_l)) - g_nl Re(e^{-i theta_nl} rho_l)]
 *   dL/dq_n = -ke sum_l c_l [Im(e^{i theta_nl} conj(A_l)) + g_nl Im(e^{-i theta_nl} rho_l)]
 * rho is over all atoms. A_l and the outputs are over the rows (all atoms when
 * rows is NULL): A_l is exact when G vanishes outside the rows. Outputs are
 * accumulated at the rows' atoms.
 */
int orc_kspace_adjoint(const orc_system* sy, const uint32_t* s, const double* q, const int64_t* rows,
                       int64_t n_rows, int32_t n_k, const int32_t* kvec, const double* wk, const double* rho,
                       const double* G, double* g_pos, double* g_q)
{
    const double L = sy->L, V = L * L * L, tpl = 2.0 * ORC_PI / L;
    double* A = (double*)calloc((size_t)(2 * n_k > 0 ? 2 * n_k : 1), sizeof(double));
    if (!A) return ORC_ENOMEM;
#pragma omp parallel for schedule(static)
    for (int32_t l = 0; l < n_k; ++l) {
        double k[3] = {tpl * kvec[3 * l], tpl * kvec[3 * l + 1], tpl * kvec[3 * l + 2]};
        double re = 0.0, im = 0.0;
        for (int64_t r = 0; r < n_rows; ++r) {
            const int64_t m = orc_row_atom(rows, r);
            double th = orc_phase(kvec + 3 * l, s + 3 * m);
            double g = G[3 * m] * k[0] + G[3 * m + 1] * k[1] + G[3 * m + 2] * k[2];
            re += q[m] * g * cos(th);
            im += q[m] * g * sin(th);
        }
        A[2 * l] = re;
        A[2 * l + 1] = im;
    }
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n_rows; ++r) {
        const int64_t i = orc_row_atom(rows, r);
        double gp[3] = {0, 0, 0}, gq = 0.0;
        for (int32_t l = 0; l < n_k; ++l) {
            double k[3] = {tpl * kvec[3 * l], tpl * kvec[3 * l + 1], tpl * kvec[3 * l + 2]};
            double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            double c = wk[l] * 4.0 * ORC_PI / (V * k2);
            double th = orc_phase(kvec + 3 * l, s + 3 * i);
            double ct = cos(th), st = sin(th);
            double g = G[3 * i] * k[0] + G[3 * i + 1] * k[1] + G[3 * i + 2] * k[2];
            /* e^{i th} conj(A) = (ct + i st)(Ar - i Ai) */
            double eA_re = ct * A[2 * l] + st * A[2 * l + 1];
            double eA_im = st * A[2 * l] - ct * A[2 * l + 1];
            /* e^{-i th} rho = (ct - i st)(rr + i ri) */
            double er_re = ct * rho[2 * l] + st * rho[2 * l + 1];
            double er_im = ct * rho[2 * l + 1] - st * rho[2 * l];
            double t = c * (eA_re - g * er_re);
            for (int a = 0; a < 3; ++a) gp[a] += t * k[a];
            gq += c * (eA_im + g * er_im);
        }
        for (int a = 0; a < 3; ++a) g_pos[3 * i + a] += -sy->ke * q[i] * gp[a];
        if (g_q) g_q[i] += -sy->ke * gq;
    }
    free(A);
    return ORC_OK;
}

/* Batches of a set of rows (Algorithm 1: p~ shell members per atom, or all
 * when N_S <= p~): ranks per row into batch_rank at batch_off (pass 1 with
 * batch_rank == NULL writes the counts), weights w = N_S / p~ (1 when all). */
int orc_shell_batches(uint64_t seed, uint64_t step, const int64_t* rows, int64_t n_rows, const int64_t* shell_off,
                      int32_t p_s, int64_t* batch_off, int32_t* batch_rank, double* w)
{
    if (!batch_rank) {
        batch_off[0] = 0;
        for (int64_t r = 0; r < n_rows; ++r) {
            int64_t n_s = shell_off[r + 1] - shell_off[r];
            batch_off[r + 1] = batch_off[r] + (n_s <= p_s ? n_s : p_s);
        }
        return ORC_OK;
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t id = orc_row_atom(rows, r);
        int32_t n_s = (int32_t)(shell_off[r + 1] - shell_off[r]);
        orc_shell_ranks(seed, step, id, n_s, p_s, batch_rank + batch_off[r]);
        w[r] = n_s > p_s ? (double)n_s / (double)p_s : 1.0;
    }
    return ORC_OK;
}

/* Membership of list or batch entries at the positions s: accept[e] = 1 when
 * entry e of row r (the atom of rank batch_rank[e] in the row's list, or entry
 * e itself when batch_off is NULL) is a member, with the thresholds of O1:
 * kind 0: of C(i) (D^2 <= T_c); kind 1: of S(i) (T_c < D^2 <= T_s);
 * kind 2: of the full list (D^2 <= T_s); never i itself or i's molecule.
 * Used by stencil sampling (the batch is drawn from candidates) and by lists
 * built with a skin (entries may have left their set). */
int orc_batch_accept(const uint32_t* s, const int32_t* mol, double L, double r_core, double r_shell, int kind,
                     const int64_t* rows, int64_t n_rows, const int64_t* shell_off, const int32_t* shell_idx,
                     const int64_t* batch_off, const int32_t* batch_rank, uint8_t* accept)
{
    uint64_t t_core = orc_threshold(r_core, L);
    uint64_t t_shell = orc_threshold(r_shell, L);
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t i = orc_row_atom(rows, r);
        int64_t cnt = batch_off ? batch_off[r + 1] - batch_off[r] : shell_off[r + 1] - shell_off[r];
        int64_t e0 = batch_off ? batch_off[r] : shell_off[r];
        for (int64_t k = 0; k < cnt; ++k) {
            int64_t j = shell_idx[shell_off[r] + (batch_off ? batch_rank[e0 + k] : k)];
            int ok = j != i && !orc_excluded(mol, i, j);
            if (ok) {
                uint64_t d2 = orc_dist2(s, i, j);
                ok = kind == 0 ? d2 <= t_core : (kind == 1 ? d2 > t_core && d2 <= t_shell : d2 <= t_shell);
            }
            accept[e0 + k] = (uint8_t)ok;
        }
    }
    return ORC_OK;
}

/* Excluded partners of each row atom: the other atoms with the same molecule
 * id >= 0, in id order. order[] holds all atoms with mol >= 0 sorted by
 * (mol, id) and pos_in_order[i] the position of atom i in it (-1 if none).
 * Pass 1 (idx == NULL) writes the counts into off[r+1]. */
int orc_exclusion_rows(int64_t n, const int32_t* mol, const int64_t* order, int64_t n_order,
                       const int64_t* pos_in_order, const int64_t* rows, int64_t n_rows, int64_t* off, int64_t* idx)
{
    (void)n;
    if (!idx) off[0] = 0;
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t i = orc_row_atom(rows, r);
        int64_t p = pos_in_order[i];
        int64_t cnt = 0;
        if (p >= 0) {
            int64_t a = p, b = p;
            while (a > 0 && mol[order[a - 1]] == mol[i]) --a;
            while (b + 1 < n_order && mol[order[b + 1]] == mol[i]) ++b;
            for (int64_t t = a; t <= b; ++t) {
                if (order[t] == i) continue;
                if (idx) idx[off[r] + cnt] = order[t];
                ++cnt;
            }
        }
        if (!idx) off[r + 1] = off[r] + cnt;
    }
    return ORC_OK;
}

/* Threads the OpenMP loops of the oracle run on (for reporting its timing). */
int orc_num_threads(void) { return omp_get_max_threads(); }
