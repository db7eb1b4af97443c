// Host runtime behind the C ABI of include/irbe.h: argument checks, device
// memory ownership, the k-sampling table, the exclusion table, and the order of
// the kernels of one force evaluation (Algorithm 1 of Liang, Xu, Zhao,
// arXiv:2204.13595, force steps) on the handle's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "irbe_device.hpp"
#include "irbe_internal.hpp"

using namespace irbe;

// Per-call scratch of irbe_compute_forces_noalloc: one array per GPU, held
// until the process ends. Host code never passes this name to a kernel (on the
// host it only stands in for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

// Device address of `scratch` on each device, looked up once per device (with
// that device current) by the first irbe_create there.
struct ScratchAddr {
    bool looked_up = false;
    void* ptr = nullptr;
    hipError_t err = hipSuccess;
};
std::mutex g_scratch_mutex;
std::vector<ScratchAddr> g_scratch_addr;

void lookup_scratch(int device)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (device < 0) return;
    if ((size_t)device >= g_scratch_addr.size()) g_scratch_addr.resize((size_t)device + 1);
    ScratchAddr& a = g_scratch_addr[(size_t)device];
    if (a.looked_up) return;
    void* p = nullptr;
    a.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    a.ptr = a.err == hipSuccess ? p : nullptr;
    a.looked_up = true;
}

// The address found for `device`, or nullptr (err says why).
void* scratch_addr(int device, hipError_t* err)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (device < 0 || (size_t)device >= g_scratch_addr.size() || !g_scratch_addr[(size_t)device].looked_up) {
        *err = hipErrorNotInitialized;
        return nullptr;
    }
    *err = g_scratch_addr[(size_t)device].err;
    return g_scratch_addr[(size_t)device].ptr;
}

thread_local std::string g_create_error;

constexpr double kTwo32 = 4294967296.0;
constexpr double kTwo64 = 18446744073709551616.0;
constexpr double kPi = 3.14159265358979323846;
constexpr int64_t kMaxCells = int64_t(1) << 27;
constexpr int32_t kMaxM = 1 << 16;

irbe_status fail(irbe_ctx* h, irbe_status st, const std::string& msg)
{
    if (h) h->last_error = msg;
    else g_create_error = msg;
    return st;
}

irbe_status hip_fail(irbe_ctx* h, hipError_t e, const char* where)
{
    const irbe_status st = e == hipErrorOutOfMemory ? IRBE_ENOMEM : IRBE_EHIP;
    return fail(h, st, std::string(where) + ": " + hipGetErrorString(e));
}

#define IRBE_TRY(h, expr, where)                      \
    do {                                              \
        const hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess) return hip_fail(h, e_, where); \
    } while (0)

// A launcher bracketed by timing events when timing is on.
#define IRBE_STAGE(h, stage, expr, where) \
    do {                                  \
        stage_begin(h);                   \
        IRBE_TRY(h, expr, where);         \
        stage_end(h, stage);              \
    } while (0)

template <typename T>
hipError_t dalloc(irbe_ctx* h, T** p, size_t count)
{
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    h->owned.push_back(q);
    *p = (T*)q;
    return hipSuccess;
}

hipError_t dalloc_bytes(irbe_ctx* h, void** p, size_t bytes)
{
    return dalloc(h, (unsigned char**)p, bytes);
}

void dfree(irbe_ctx* h, void* p)
{
    if (!p) return;
    auto it = std::find(h->owned.begin(), h->owned.end(), p);
    if (it != h->owned.end()) h->owned.erase(it);
    hipFree(p);
}

}  // namespace

namespace irbe {

hipError_t ensure_buckets(irbe_ctx* h, int64_t records)
{
    hipError_t e = hipSuccess;
    if (!h->bk_cursor) e = dalloc(h, &h->bk_cursor, 2 * (size_t)h->geo.n_c * (size_t)h->geo.n_c);
    if (e != hipSuccess || records <= h->bk_total) return e;
    dfree(h, h->bk_c);
    dfree(h, h->bk_j);
    h->bk_c = nullptr;
    h->bk_j = nullptr;
    h->bk_total = 0;
    e = dalloc_bytes(h, &h->bk_c, 4 * (size_t)records * h->real_size);
    if (e == hipSuccess) e = dalloc(h, &h->bk_j, (size_t)records);
    if (e == hipSuccess) h->bk_total = records;
    return e;
}

hipError_t ensure_draw_bits(irbe_ctx* h, size_t words)
{
    if (h->draw_bits_words >= words) return hipSuccess;
    dfree(h, h->draw_bits);
    h->draw_bits = nullptr;
    h->draw_bits_words = 0;
    const hipError_t e = dalloc(h, &h->draw_bits, words);
    if (e == hipSuccess) h->draw_bits_words = words;
    return e;
}

hipError_t ensure_batch_atoms(irbe_ctx* h)
{
    if (h->batch_j) return hipSuccess;
    return dalloc(h, &h->batch_j, (size_t)h->cfg.n_atoms * (size_t)h->p_stride);
}

}  // namespace irbe

namespace {

// Quantized-geometry constants, in the FP64 operation order that fixes them:
// n_c = floor(L / (r_core + skin)), R = floor((r_shell + skin) n_c / L) + 1,
// T(r) = floor(t * t) with t = r 2^32 / L.
void geometry(const irbe_config& c, Geometry& g)
{
#pragma clang fp contract(off)
    const double L = c.box_length;
    const double rc_l = c.r_core + c.skin, rs_l = c.r_shell + c.skin;
    g.n_c = (int32_t)std::floor(L / rc_l);
    g.reach = (int32_t)std::floor(rs_l * (double)g.n_c / L) + 1;
    if (2 * g.reach + 1 <= g.n_c) {
        g.lo = -g.reach;
        g.hi = g.reach;
    } else {
        g.lo = -((g.n_c - 1) / 2);
        g.hi = g.lo + g.n_c - 1;
    }
    auto threshold = [L](double r) {
        const double t = r * kTwo32 / L;
        return (uint64_t)std::floor(t * t);
    };
    g.t_core = threshold(c.r_core);
    g.t_shell = threshold(c.r_shell);
    g.skin = c.skin > 0.0;
    g.tl_core = threshold(rc_l);
    g.tl_lo = !g.skin ? g.t_core : (c.r_core > c.skin ? threshold(c.r_core - c.skin) : 0);
    g.tl_shell = threshold(rs_l);
    g.inv_l = 1.0 / L;
    g.quantum = L / kTwo32;
    g.n_cells = (int64_t)g.n_c * g.n_c * g.n_c;
}

// Per-axis inverse-CDF table of the discrete Gaussian w(m) = exp(-(pi m/(beta L))^2)
// (Eqs. (2.6)-(2.8)): M = smallest m >= 0 with w(m+1) < 2^-64,
// H = sum_{m=-M..M} w(m) in ascending m, S = H^3 - 1,
// U[m+M] = floor(2^64 cdf(m)) with the cdf accumulated in ascending m, U[2M] = 2^64-1.
int32_t ktable(double beta, double L, std::vector<uint64_t>& U, double& H, double& S)
{
#pragma clang fp contract(off)
    const double a = kPi / (beta * L);
    auto w = [a](int32_t m) {
        const double x = a * (double)m;
        return std::exp(-(x * x));
    };
    int32_t M = 0;
    while (w(M + 1) >= 1.0 / kTwo64) {
        ++M;
        if (M > kMaxM) return -1;
    }
    H = 0.0;
    for (int32_t m = -M; m <= M; ++m) H += w(m);
    U.assign(2 * (size_t)M + 1, 0);
    double c = 0.0;
    for (int32_t m = -M; m <= M; ++m) {
        c += w(m);
        const double x = (c / H) * kTwo64;
        U[m + M] = (x >= kTwo64) ? UINT64_MAX : (uint64_t)x;
    }
    U[2 * M] = UINT64_MAX;
    S = H * H * H - 1.0;
    return M;
}

int32_t round_up32(double v) { return (int32_t)((std::ceil(v) + 31.0) / 32.0) * 32; }

// Rows of cap_core and cap_shell entries per atom; shell entries of 2 bytes
// (16-bit codes) while the handle can use them, else 4.
hipError_t alloc_lists(irbe_ctx* h, int32_t cap_core, int32_t cap_shell)
{
    const size_t n = (size_t)h->cfg.n_atoms;
    dfree(h, h->core);
    dfree(h, h->shell);
    h->core = h->shell = nullptr;
    hipError_t e = dalloc(h, &h->core, n * (size_t)cap_core);
    if (e != hipSuccess) return e;
    const int32_t eb = h->shell16_ok && h->sgroup != nullptr && irbe::shell16_possible(h) ? 2 : 4;
    e = dalloc(h, &h->shell, (n * (size_t)cap_shell * eb + 3) / 4);
    if (e != hipSuccess) return e;
    h->shell_bytes = eb;
    h->cap_core = cap_core;
    h->cap_shell = cap_shell;
    return hipSuccess;
}

// Shell rows of 4-byte entries once the 16-bit codes have been given up
// (after the queued work that may still read the old rows).
hipError_t ensure_shell_rows_32(irbe_ctx* h)
{
    if (h->shell_bytes == 4 || h->shell16_ok) return hipSuccess;
    const hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
    h->have_lists = false;
    return alloc_lists(h, h->cap_core, h->cap_shell);
}

// Rows for lists of the given longest lengths, grown by at least 30% so that a
// few rounds converge (waits: the old rows may still be read by queued work).
hipError_t grow_lists(irbe_ctx* h, int32_t max_core, int32_t max_shell)
{
    const int32_t nc = max_core > h->cap_core
                           ? std::max(round_up32(1.15 * max_core + 32.0), round_up32(1.3 * h->cap_core))
                           : h->cap_core;
    const int32_t ns = !h->stencil && max_shell > h->cap_shell
                           ? std::max(round_up32(1.15 * max_shell + 32.0), round_up32(1.3 * h->cap_shell))
                           : h->cap_shell;
    if (nc == h->cap_core && ns == h->cap_shell) return hipSuccess;
    if (ns > 65535) return hipErrorInvalidValue;
    const hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
    h->have_lists = false;
    return alloc_lists(h, nc, ns);
}

// Sorted index of the 16-bit shell entry e of an atom of list-build group grp,
// decoded on the host (cs: the cell starts of the build); the layout of the
// codes is that of ListCode. Clamped to [0, N) as on the device.
int32_t decode_shell_entry(const ListCode& lc, const std::vector<int32_t>& cs, int32_t grp, uint32_t e)
{
    if (grp < 0 || grp >= lc.gpr * lc.n_c * lc.n_c) return 0;
    auto wrap = [&](int c) { return c < 0 ? c + lc.n_c : (c >= lc.n_c ? c - lc.n_c : c); };
    const int rid = (int)(e >> lc.pb), p = (int)(e & ((1u << lc.pb) - 1));
    if (rid >= lc.span * lc.span) return 0;
    const int rowid = grp / lc.gpr;
    const int cz = rowid / lc.n_c, cy = rowid % lc.n_c;
    const int x0 = (grp % lc.gpr) * lc.G;
    const int span_u = std::min(lc.G, lc.n_c - x0) - 1 + lc.span;
    const int xu0 = wrap(x0 + lc.lo);
    const int lenA = std::min(span_u, lc.n_c - xu0);
    const int z = wrap(cz + rid / lc.span + lc.lo), y = wrap(cy + rid % lc.span + lc.lo);
    const int64_t row = ((int64_t)z * lc.n_c + y) * lc.n_c;
    const int32_t a = cs[row + xu0], na = cs[row + xu0 + lenA] - a;
    const int64_t j = p < na ? (int64_t)a + p : (int64_t)cs[row] + (p - na);
    return (int32_t)std::min<int64_t>(std::max<int64_t>(j, 0), cs.back() - 1);
}

irbe_status check_device_error(irbe_ctx* h)
{
    uint32_t err = 0;
    int32_t mx[2] = {0, 0};
    IRBE_TRY(h, hipMemcpyAsync(&err, h->err, sizeof(err), hipMemcpyDeviceToHost, h->stream), "read error word");
    IRBE_TRY(h, hipMemcpyAsync(mx, h->maxcnt, sizeof(mx), hipMemcpyDeviceToHost, h->stream), "read list sizes");
    IRBE_TRY(h, hipStreamSynchronize(h->stream), "synchronize");
    if (err) {
        IRBE_TRY(h, launch_fill_i32(h->stream, (int32_t*)h->err, 0, 1), "clear error word");
        if (err & ERR_NONFINITE) return fail(h, IRBE_ENONFINITE, "non-finite position");
        // a stencil row's candidates beyond the 16-bit entry codes: 32-bit entries
        // from the next build on
        if (err & ERR_SHELL_CODE) h->shell16_ok = false;
        // the rows of some build since the last check were too short: the forces
        // computed from those lists miss entries; grow the rows for the next build
        const hipError_t e = grow_lists(h, std::max(mx[0], h->max_core), std::max(mx[1], h->max_shell));
        if (e == hipErrorInvalidValue) return fail(h, IRBE_ECAPACITY, "more than 65535 list entries per atom");
        if (e != hipSuccess) return hip_fail(h, e, "grow lists");
        if (err & ERR_SHELL_CODE)
            return fail(h, IRBE_ECAPACITY,
                        "a shell stencil row's candidates exceeded the 16-bit entry codes in a build since the last "
                        "check: forces computed from those lists are wrong; 32-bit entries from now on, build the "
                        "lists again");
        return fail(h, IRBE_ECAPACITY,
                    "list capacity exceeded by a build since the last check: forces computed from those lists are "
                    "incomplete; the rows have been grown, build the lists again");
    }
    return IRBE_OK;
}

// Reads back, without waiting, the error word and list lengths of the last
// asynchronous build once its copy has completed; grows the rows when they
// were too short (the error stays set for the next waiting call to report).
irbe_status poll_list_check(irbe_ctx* h)
{
    if (!h->chk_pending) return IRBE_OK;
    const hipError_t q = hipEventQuery(h->chk_event);
    if (q == hipErrorNotReady) return IRBE_OK;
    if (q != hipSuccess) return hip_fail(h, q, "list check");
    h->chk_pending = false;
    const uint32_t err = (uint32_t)h->chk_host[0];
    h->max_core = h->chk_host[1];
    h->max_shell = h->chk_host[2];
    // (an overflowing code: 32-bit entries from the next build on)
    if (err & ERR_SHELL_CODE) h->shell16_ok = false;
    if (err & (ERR_CORE_CAP | ERR_SHELL_CAP)) {
        const hipError_t e = grow_lists(h, h->max_core, h->max_shell);
        if (e == hipErrorInvalidValue) return fail(h, IRBE_ECAPACITY, "more than 65535 list entries per atom");
        if (e != hipSuccess) return hip_fail(h, e, "grow lists");
    }
    return IRBE_OK;
}

void stage_begin(irbe_ctx* h)
{
    if (!h->timing) return;
    hipEventCreate(&h->open_start);
    hipEventRecord(h->open_start, h->stream);
}

void stage_end(irbe_ctx* h, int stage)
{
    if (!h->timing || !h->open_start) return;
    hipEvent_t stop;
    hipEventCreate(&stop);
    hipEventRecord(stop, h->stream);
    h->pending.push_back({stage, h->open_start, stop});
    h->open_start = nullptr;
}

void drain_timing(irbe_ctx* h)
{
    for (auto& p : h->pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(p.stop) == hipSuccess && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
            h->stage_ms[p.stage] += ms;
            h->stage_n[p.stage] += 1;
        }
        hipEventDestroy(p.start);
        hipEventDestroy(p.stop);
    }
    h->pending.clear();
}

template <typename real>
void lj_tables(const irbe_ctx* h, std::vector<LJ<real>>& tab, std::vector<real>& raw)
{
    const int nt2 = h->cfg.n_types * h->cfg.n_types;
    tab.resize(nt2);
    raw.resize(2 * (size_t)nt2);
    for (int t = 0; t < nt2; ++t) {
        const double s = h->lj_sigma_host[t], e = h->lj_eps_host[t];
        const double s6 = s * s * s * s * s * s;
        const double s12 = s6 * s6;
        tab[t].a12 = (real)(48.0 * e * s12);
        tab[t].b6 = (real)(24.0 * e * s6);
        tab[t].c12 = (real)(4.0 * e * s12);
        tab[t].c6 = (real)(4.0 * e * s6);
        const double k = h->cfg.lj_cut;
        tab[t].rc2 = k > 0.0 ? (real)(k * s * k * s) : std::numeric_limits<real>::max();
        tab[t].esh = k > 0.0 ? (real)(4.0 * e * (std::pow(k, -12.0) - std::pow(k, -6.0))) : (real)0;
        raw[t] = (real)s;
        raw[nt2 + t] = (real)e;
    }
}

irbe_status upload_lj(irbe_ctx* h)
{
    const int nt2 = h->cfg.n_types * h->cfg.n_types;
    if (h->fp64) {
        std::vector<LJ<double>> tab;
        std::vector<double> raw;
        lj_tables(h, tab, raw);
        IRBE_TRY(h, hipMemcpyAsync(h->lj, tab.data(), sizeof(LJ<double>) * nt2, hipMemcpyHostToDevice, h->stream),
                 "upload LJ");
        IRBE_TRY(h, hipMemcpyAsync(h->lj_raw, raw.data(), sizeof(double) * 2 * nt2, hipMemcpyHostToDevice, h->stream),
                 "upload LJ");
        IRBE_TRY(h, hipStreamSynchronize(h->stream), "upload LJ");
    } else {
        std::vector<LJ<float>> tab;
        std::vector<float> raw;
        lj_tables(h, tab, raw);
        IRBE_TRY(h, hipMemcpyAsync(h->lj, tab.data(), sizeof(LJ<float>) * nt2, hipMemcpyHostToDevice, h->stream),
                 "upload LJ");
        IRBE_TRY(h, hipMemcpyAsync(h->lj_raw, raw.data(), sizeof(float) * 2 * nt2, hipMemcpyHostToDevice, h->stream),
                 "upload LJ");
        IRBE_TRY(h, hipStreamSynchronize(h->stream), "upload LJ");
    }
    return IRBE_OK;
}

bool set_lj_host(irbe_ctx* h, const double* sig, const double* eps, std::string& why)
{
    const int nt2 = h->cfg.n_types * h->cfg.n_types;
    std::vector<double> s(sig, sig + nt2), e(eps, eps + nt2);
    for (int t = 0; t < nt2; ++t)
        if (!std::isfinite(s[t]) || !std::isfinite(e[t]) || s[t] < 0.0) {
            why = "LJ tables must be finite with sigma >= 0";
            return false;
        }
    h->lj_sigma_host = s;
    h->lj_eps_host = e;
    return true;
}

}  // namespace

extern "C" {

irbe_status irbe_create(const irbe_config* cfg, void* hip_stream, irbe_handle* out)
{
    if (!cfg || !out) return fail(nullptr, IRBE_EINVAL, "null argument");
    *out = nullptr;
    const irbe_config& c = *cfg;
    if (c.abi_version != IRBE_ABI_VERSION) return fail(nullptr, IRBE_EINVAL, "abi_version mismatch");
    if (c.precision != IRBE_MIXED_FP32 && c.precision != IRBE_FP64) return fail(nullptr, IRBE_EINVAL, "bad precision");
    if (c.n_atoms < 1 || c.n_atoms > (int64_t(1) << 30)) return fail(nullptr, IRBE_EINVAL, "n_atoms out of range");
    if (!(c.box_length > 0.0) || !std::isfinite(c.box_length)) return fail(nullptr, IRBE_EINVAL, "bad box_length");
    if (!(c.ewald_beta > 0.0) || !std::isfinite(c.ewald_beta)) return fail(nullptr, IRBE_EINVAL, "bad ewald_beta");
    if (!std::isfinite(c.coulomb_k)) return fail(nullptr, IRBE_EINVAL, "bad coulomb_k");
    if (!(c.r_core > 0.0) || !(c.r_shell > c.r_core) || !(c.r_shell < 0.5 * c.box_length))
        return fail(nullptr, IRBE_EINVAL, "need 0 < r_core < r_shell < L/2");
    if (c.p_kspace < 1) return fail(nullptr, IRBE_EINVAL, "p_kspace must be >= 1");
    if (c.n_types < 1 || c.n_types > 16) return fail(nullptr, IRBE_EINVAL, "n_types must be in 1..16");
    if (!(c.capacity_hint >= 0.0) || !std::isfinite(c.capacity_hint))
        return fail(nullptr, IRBE_EINVAL, "bad capacity_hint");
    if (!(c.skin >= 0.0) || !std::isfinite(c.skin) || !(c.r_shell + c.skin < 0.5 * c.box_length))
        return fail(nullptr, IRBE_EINVAL, "need skin >= 0 and r_shell + skin < L/2");
    if (!(c.lj_cut >= 0.0) || !std::isfinite(c.lj_cut)) return fail(nullptr, IRBE_EINVAL, "need lj_cut >= 0");
    if (c.shell_source != IRBE_SHELL_LIST && c.shell_source != IRBE_SHELL_STENCIL)
        return fail(nullptr, IRBE_EINVAL, "bad shell_source");
    if (c.shell_source == IRBE_SHELL_STENCIL && c.p_shell <= 0)
        return fail(nullptr, IRBE_EINVAL, "stencil sampling needs p_shell > 0");
    if (c.shell_entries != IRBE_ENTRIES_AUTO && c.shell_entries != IRBE_ENTRIES_32)
        return fail(nullptr, IRBE_EINVAL, "bad shell_entries");

    irbe_ctx* h = new (std::nothrow) irbe_ctx();
    if (!h) return fail(nullptr, IRBE_ENOMEM, "host allocation failed");
    h->cfg = c;
    h->stream = (hipStream_t)hip_stream;
    h->fp64 = c.precision == IRBE_FP64;
    h->real_size = h->fp64 ? 8 : 4;
    h->full_list = c.p_shell <= 0;
    h->stencil = c.shell_source == IRBE_SHELL_STENCIL;
    h->shell16_ok = c.shell_entries == IRBE_ENTRIES_AUTO;
    geometry(c, h->geo);
    if (h->geo.n_c < 3) {
        delete h;
        return fail(nullptr, IRBE_EINVAL, "floor(L / (r_core + skin)) must be >= 3");
    }
    if (h->stencil && (h->geo.hi - h->geo.lo + 1) * (h->geo.hi - h->geo.lo + 1) > 128) {
        delete h;
        return fail(nullptr, IRBE_EUNSUPPORTED, "stencil sampling supports at most 128 stencil rows");
    }
    if (h->geo.hi - h->geo.lo + 1 > 191) {
        delete h;
        return fail(nullptr, IRBE_EUNSUPPORTED, "shell stencils wider than 191 cells per axis");
    }
    if (h->geo.n_cells > kMaxCells || h->geo.n_c > 1000) {
        delete h;
        return fail(nullptr, IRBE_EUNSUPPORTED, "too many cells");
    }
    std::vector<uint64_t> U;
    h->kM = ktable(c.ewald_beta, c.box_length, U, h->kH, h->kS);
    if (h->kM < 0) {
        delete h;
        return fail(nullptr, IRBE_EUNSUPPORTED, "k table too large (beta L too big)");
    }
    hipError_t e = hipGetDevice(&h->device);
    if (e == hipSuccess) lookup_scratch(h->device);
    const size_t n = (size_t)c.n_atoms;
    const size_t rs = h->real_size;
    const int64_t nb = blocks_for(c.n_atoms, kBlock);
    // per-block partial buffers must cover the largest grid of any pair kernel:
    // 64-thread blocks of the thread-per-atom kernels and the cooperative kernels'
    // blocks of four wavefronts with two or more atoms each
    // (the bucketed pair adjoint runs blocks of as few as 8 atoms)
    const int64_t nb64 = std::max(blocks_for(c.n_atoms, 64), blocks_for(c.n_atoms, 8));
    const int64_t nbr = rho_blocks(c.n_atoms);
    const size_t P = (size_t)c.p_kspace;
    const int nt2 = c.n_types * c.n_types;
#define ALLOC(expr)                      \
    if (e == hipSuccess) e = (expr);
    ALLOC(dalloc(h, &h->err, 1));
    ALLOC(dalloc(h, &h->maxcnt, 2));
    ALLOC(dalloc(h, &h->adj_atomics, 1));
    ALLOC(dalloc(h, &h->ktab, U.size()));
    ALLOC(dalloc_bytes(h, &h->q_orig, n * rs));
    ALLOC(dalloc(h, &h->type_orig, n));
    ALLOC(dalloc(h, &h->mol_orig, n));
    ALLOC(dalloc_bytes(h, &h->lj, (size_t)nt2 * (h->fp64 ? sizeof(LJ<double>) : sizeof(LJ<float>))));
    ALLOC(dalloc_bytes(h, &h->lj_raw, (size_t)nt2 * 2 * rs));
    ALLOC(dalloc(h, &h->sumq2, 1));
    ALLOC(dalloc(h, &h->q2part, (size_t)nb));
    ALLOC(dalloc(h, &h->sq, n));
    ALLOC(dalloc(h, &h->cell_count, (size_t)h->geo.n_cells));
    ALLOC(dalloc(h, &h->cell_start, (size_t)h->geo.n_cells + 1));
    ALLOC(dalloc(h, &h->cell_bound, (size_t)h->geo.n_c + 1));
    {
        int64_t m = h->geo.n_cells;
        do {
            m = blocks_for(m, 1024);
            int32_t* lv = nullptr;
            ALLOC(dalloc(h, &lv, (size_t)m + 1));
            h->scan_levels.push_back(lv);
        } while (m > 1);
        int32_t* lv = nullptr;
        ALLOC(dalloc(h, &lv, 2));
        h->scan_levels.push_back(lv);
    }
    ALLOC(dalloc(h, &h->perm, n));
    ALLOC(dalloc(h, &h->rank, n));
    ALLOC(dalloc(h, &h->spos, n));
    ALLOC(dalloc(h, &h->spk, n));
    if (!h->fp64) ALLOC(dalloc(h, &h->spq, n));
    if (h->geo.skin) ALLOC(dalloc(h, &h->brow, n));
    ALLOC(dalloc_bytes(h, &h->sq_r, n * rs));
    ALLOC(dalloc(h, &h->smol, n));
    ALLOC(dalloc(h, &h->sxr, n));
    ALLOC(dalloc(h, &h->ncore, n));
    h->p_stride = c.p_shell > 0 ? (c.p_shell + 3) / 4 * 4 : 0;
    if (h->p_stride > 0) ALLOC(dalloc(h, &h->ranks, n * (size_t)h->p_stride));
    if (h->stencil) ALLOC(dalloc(h, &h->scell, n));
    if (!h->full_list && !h->stencil && h->shell16_ok) ALLOC(dalloc(h, &h->sgroup, n));
    ALLOC(dalloc(h, &h->nshell, n));
    ALLOC(dalloc_bytes(h, &h->fsr, 3 * n * rs));
    ALLOC(dalloc(h, &h->pair_part, (size_t)nb64 * kPairPartials));
    h->part_blocks = nb64;
    ALLOC(dalloc(h, &h->fcorr, 3));
    ALLOC(dalloc(h, &h->pair_slices, 256 * 12));
    ALLOC(dalloc(h, &h->ev_pair, kPairPartials));
    ALLOC(dalloc(h, &h->kvec, P));
    ALLOC(dalloc(h, &h->kcoef, 4 * P));
    ALLOC(dalloc(h, &h->rho_part, 4 * P * (size_t)nbr));
    ALLOC(dalloc(h, &h->rho, 2 * P));
    ALLOC(dalloc(h, &h->Avec, 2 * P));
    ALLOC(dalloc_bytes(h, &h->kforce, P * sizeof(KForce<double>)));
    ALLOC(dalloc_bytes(h, &h->kadj, P * sizeof(KAdj<double>)));
    ALLOC(dalloc_bytes(h, &h->gs, 3 * n * rs));
    ALLOC(dalloc(h, &h->gpart, (size_t)nb * 3));
    ALLOC(dalloc(h, &h->gmean, 3));
    ALLOC(dalloc_bytes(h, &h->gself, 3 * n * rs));
    ALLOC(dalloc_bytes(h, &h->gscat, 3 * n * rs));
    ALLOC(dalloc_bytes(h, &h->gqself, n * rs));
    ALLOC(dalloc_bytes(h, &h->gqscat, n * rs));
    ALLOC(dalloc(h, &h->ljpart, (size_t)nb64 * 2 * kMaxTypesGrad * kMaxTypesGrad));
    ALLOC(dalloc(h, &h->lj_slices, 256 * 2 * kMaxTypesGrad * kMaxTypesGrad));
#undef ALLOC
    if (e == hipSuccess) {
        const double L = c.box_length;
        const double rho_n = (double)c.n_atoms / (L * L * L);
        auto ball = [](double r) { return 4.0 / 3.0 * kPi * r * r * r; };
        const double vc = ball(c.r_core + c.skin);
        const double vlo = ball(std::max(c.r_core - c.skin, 0.0));
        const double vs = ball(c.r_shell + c.skin);
        int32_t cap_c = round_up32(1.3 * rho_n * vc + 32.0);
        int32_t cap_s = round_up32(1.3 * rho_n * (h->full_list ? vs : vs - vlo) + 32.0);
        if (c.capacity_hint > 0.0) cap_s = round_up32(c.capacity_hint);
        if (h->full_list) cap_c = 1;
        if (h->stencil) cap_s = 1;  // no shell list
        cap_c = (int32_t)std::min<int64_t>(cap_c, c.n_atoms + 32);
        cap_s = (int32_t)std::min<int64_t>(cap_s, c.n_atoms + 32);
        e = alloc_lists(h, cap_c, cap_s);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->ktab, U.data(), U.size() * sizeof(uint64_t), hipMemcpyHostToDevice, h->stream);
    std::vector<uint32_t> bound((size_t)h->geo.n_c + 1);
    for (int32_t c = 0; c <= h->geo.n_c; ++c)
        bound[c] = (uint32_t)((((uint64_t)c << 32) + (uint64_t)h->geo.n_c - 1) / (uint64_t)h->geo.n_c);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->cell_bound, bound.data(), bound.size() * 4, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipHostMalloc((void**)&h->chk_host, 4 * sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->chk_event, hipEventDisableTiming);
    if (e == hipSuccess) e = launch_fill_i32(h->stream, (int32_t*)h->err, 0, 1);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        const irbe_status st = hip_fail(nullptr, e, "irbe_create");
        irbe_destroy(h);
        return st;
    }
    *out = h;
    return IRBE_OK;
}

irbe_status irbe_set_system(irbe_handle h, const int32_t* type, const void* charge, const int32_t* molecule,
                            const double* lj_sigma_host, const double* lj_eps_host)
{
    if (!h) return IRBE_EINVAL;
    if (!type || !charge || !molecule || !lj_sigma_host || !lj_eps_host)
        return fail(h, IRBE_EINVAL, "irbe_set_system: null argument");
    std::string why;
    std::vector<double> keep_s = h->lj_sigma_host, keep_e = h->lj_eps_host;
    if (!set_lj_host(h, lj_sigma_host, lj_eps_host, why)) return fail(h, IRBE_EINVAL, why);
    const size_t n = (size_t)h->cfg.n_atoms;
    std::vector<int32_t> t(n), mol(n);
    IRBE_TRY(h, hipMemcpyAsync(t.data(), type, n * 4, hipMemcpyDeviceToHost, h->stream), "read types");
    IRBE_TRY(h, hipMemcpyAsync(mol.data(), molecule, n * 4, hipMemcpyDeviceToHost, h->stream), "read molecules");
    IRBE_TRY(h, hipStreamSynchronize(h->stream), "set_system");
    for (size_t i = 0; i < n; ++i)
        if (t[i] < 0 || t[i] >= h->cfg.n_types) {
            h->lj_sigma_host = keep_s;
            h->lj_eps_host = keep_e;
            return fail(h, IRBE_EINVAL, "atom type out of range");
        }
    // exclusion partners: the other atoms with the same molecule id >= 0, by id
    std::vector<std::pair<int32_t, int32_t>> order;
    order.reserve(n);
    for (size_t i = 0; i < n; ++i)
        if (mol[i] >= 0) order.emplace_back(mol[i], (int32_t)i);
    std::sort(order.begin(), order.end());
    std::vector<int32_t> off(n + 1, 0);
    for (size_t a = 0; a < order.size();) {
        size_t b = a;
        while (b < order.size() && order[b].first == order[a].first) ++b;
        if (b - a > 4096) return fail(h, IRBE_EUNSUPPORTED, "molecules of more than 4096 atoms");
        for (size_t k = a; k < b; ++k) off[order[k].second + 1] = (int32_t)(b - a - 1);
        a = b;
    }
    int64_t total = 0;
    for (size_t i = 0; i < n; ++i) {
        total += off[i + 1];
        if (total > INT32_MAX) return fail(h, IRBE_EUNSUPPORTED, "too many excluded pairs");
        off[i + 1] = (int32_t)total;
    }
    std::vector<int32_t> idx((size_t)std::max<int64_t>(total, 1));
    for (size_t a = 0; a < order.size();) {
        size_t b = a;
        while (b < order.size() && order[b].first == order[a].first) ++b;
        for (size_t k = a; k < b; ++k) {
            int32_t w = off[order[k].second];
            for (size_t u = a; u < b; ++u)
                if (u != k) idx[w++] = order[u].second;
        }
        a = b;
    }
    dfree(h, h->xoff);
    dfree(h, h->xidx);
    dfree(h, h->sxidx);
    h->xoff = h->xidx = h->sxidx = nullptr;
    IRBE_TRY(h, dalloc(h, &h->xoff, n + 1), "alloc exclusions");
    IRBE_TRY(h, dalloc(h, &h->xidx, idx.size()), "alloc exclusions");
    IRBE_TRY(h, dalloc(h, &h->sxidx, idx.size()), "alloc exclusions");
    h->n_excl = total;
    IRBE_TRY(h, hipMemcpyAsync(h->xoff, off.data(), (n + 1) * 4, hipMemcpyHostToDevice, h->stream), "upload");
    IRBE_TRY(h, hipMemcpyAsync(h->xidx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice, h->stream), "upload");
    IRBE_TRY(h, hipMemcpyAsync(h->type_orig, type, n * 4, hipMemcpyDeviceToDevice, h->stream), "copy types");
    IRBE_TRY(h, hipMemcpyAsync(h->mol_orig, molecule, n * 4, hipMemcpyDeviceToDevice, h->stream), "copy molecules");
    IRBE_TRY(h, hipMemcpyAsync(h->q_orig, charge, n * h->real_size, hipMemcpyDeviceToDevice, h->stream),
             "copy charges");
    IRBE_TRY(h, launch_sum_q2(h), "sum q^2");
    const irbe_status st = upload_lj(h);
    if (st != IRBE_OK) return st;
    h->have_system = true;
    h->have_lists = false;
    return IRBE_OK;
}

irbe_status irbe_update_parameters(irbe_handle h, const void* charge, const double* lj_sigma_host,
                                   const double* lj_eps_host)
{
    if (!h) return IRBE_EINVAL;
    if (!h->have_system) return fail(h, IRBE_ESTATE, "irbe_update_parameters before irbe_set_system");
    if ((lj_sigma_host == nullptr) != (lj_eps_host == nullptr))
        return fail(h, IRBE_EINVAL, "give both LJ tables or neither");
    if (lj_sigma_host) {
        std::string why;
        if (!set_lj_host(h, lj_sigma_host, lj_eps_host, why)) return fail(h, IRBE_EINVAL, why);
        const irbe_status st = upload_lj(h);
        if (st != IRBE_OK) return st;
    }
    if (charge) {
        IRBE_TRY(h, hipMemcpyAsync(h->q_orig, charge, (size_t)h->cfg.n_atoms * h->real_size, hipMemcpyDeviceToDevice,
                                   h->stream),
                 "copy charges");
        IRBE_TRY(h, launch_sum_q2(h), "sum q^2");
    }
    return IRBE_OK;
}

irbe_status irbe_build_lists(irbe_handle h, const void* pos, uint64_t step)
{
    (void)step;
    if (!h) return IRBE_EINVAL;
    if (!pos) return fail(h, IRBE_EINVAL, "irbe_build_lists: null positions");
    if (!h->have_system) return fail(h, IRBE_ESTATE, "irbe_build_lists before irbe_set_system");
    h->have_lists = false;
    h->ranks_valid = false;
    h->batch_j_valid = h->batch_j_fwd = false;
    if (h->lists_sized && !h->stencil) {
        // steady state: queue the build and a copy of its error word and list
        // lengths, and take in an earlier copy if it has completed; no wait
        const irbe_status st = poll_list_check(h);
        if (st != IRBE_OK) return st;
        IRBE_TRY(h, ensure_shell_rows_32(h), "reallocate the shell rows");
        IRBE_STAGE(h, IRBE_STAGE_BIN, launch_bin(h, pos), "binning");
        IRBE_TRY(h, launch_fill_i32(h->stream, h->maxcnt, 0, 2), "list build");
        IRBE_STAGE(h, IRBE_STAGE_LISTS, launch_build_lists(h), "list build");
        IRBE_TRY(h, hipMemcpyAsync(h->chk_host, h->err, 4, hipMemcpyDeviceToHost, h->stream), "list check");
        IRBE_TRY(h, hipMemcpyAsync(h->chk_host + 1, h->maxcnt, 8, hipMemcpyDeviceToHost, h->stream), "list check");
        IRBE_TRY(h, hipEventRecord(h->chk_event, h->stream), "list check");
        h->chk_pending = true;
        h->have_lists = true;
        return IRBE_OK;
    }
    // the first build (and every build with stencil sampling, whose stencil
    // counts size the batch draw): wait for the list lengths and grow the rows
    IRBE_STAGE(h, IRBE_STAGE_BIN, launch_bin(h, pos), "binning");
    for (int attempt = 0; attempt < 4; ++attempt) {
        IRBE_TRY(h, ensure_shell_rows_32(h), "reallocate the shell rows");
        IRBE_TRY(h, launch_fill_i32(h->stream, h->maxcnt, 0, 2), "list build");
        IRBE_STAGE(h, IRBE_STAGE_LISTS, launch_build_lists(h), "list build");
        int32_t mx[2] = {0, 0};
        uint32_t err = 0;
        IRBE_TRY(h, hipMemcpyAsync(mx, h->maxcnt, sizeof(mx), hipMemcpyDeviceToHost, h->stream), "read list sizes");
        IRBE_TRY(h, hipMemcpyAsync(&err, h->err, sizeof(err), hipMemcpyDeviceToHost, h->stream), "read error word");
        IRBE_TRY(h, hipStreamSynchronize(h->stream), "synchronize");
        if (err) {
            IRBE_TRY(h, launch_fill_i32(h->stream, (int32_t*)h->err, 0, 1), "clear error word");
            if (err & ERR_NONFINITE) return fail(h, IRBE_ENONFINITE, "non-finite position");
            // capacity bits of this build: the rows grow below and the lists are built again
            if (err & ERR_SHELL_CODE) {
                // a stencil row's candidate range too long for the 16-bit codes:
                // 32-bit entries from now on, and the lists built again
                h->shell16_ok = false;
                continue;
            }
        }
        if (h->stencil && mx[1] > 65535)
            return fail(h, IRBE_EUNSUPPORTED, "more than 65535 atoms in a shell stencil");
        if (mx[0] <= h->cap_core && (h->stencil || mx[1] <= h->cap_shell)) {
            h->max_core = mx[0];
            h->max_shell = mx[1];
            h->have_lists = true;
            h->lists_sized = true;
            return IRBE_OK;
        }
        const int32_t nc = std::max(h->cap_core, round_up32(1.15 * mx[0] + 32.0));
        const int32_t ns = h->stencil ? h->cap_shell : std::max(h->cap_shell, round_up32(1.15 * mx[1] + 32.0));
        if (ns > 65535) return fail(h, IRBE_ECAPACITY, "more than 65535 list entries per atom");
        IRBE_TRY(h, alloc_lists(h, nc, ns), "grow lists");
    }
    return fail(h, IRBE_ECAPACITY, "list capacity did not converge");
}

irbe_status irbe_compute_forces(irbe_handle h, const void* pos, uint64_t step, void* force, uint32_t flags,
                                double* energy_virial)
{
    if (!h) return IRBE_EINVAL;
    if (!pos || !force) return fail(h, IRBE_EINVAL, "irbe_compute_forces: null argument");
    if (flags & ~(uint32_t)(IRBE_ENERGY | IRBE_VIRIAL)) return fail(h, IRBE_EINVAL, "unknown flags");
    if (flags && !energy_virial) return fail(h, IRBE_EINVAL, "energy/virial requested without a buffer");
    if (!h->have_lists) return fail(h, IRBE_ESTATE, "irbe_compute_forces before irbe_build_lists");
    const bool ev = flags != 0;
    IRBE_STAGE(h, IRBE_STAGE_QUANTIZE, launch_requantize(h, pos), "quantize");
    IRBE_STAGE(h, IRBE_STAGE_KSAMPLE, launch_ksample(h, step), "k sampling");
    IRBE_STAGE(h, IRBE_STAGE_RHO, launch_rho(h, nullptr, false), "structure factor");
    IRBE_STAGE(h, IRBE_STAGE_PAIR, launch_pair_forces(h, step, ev), "pair forces");
    IRBE_STAGE(h, IRBE_STAGE_PAIR_REDUCE, launch_pair_reduce(h), "pair reduction");
    IRBE_STAGE(h, IRBE_STAGE_KSPACE, launch_kspace_forces(h, force), "k-space forces");
    if (ev) IRBE_STAGE(h, IRBE_STAGE_ENERGY, launch_energy_finalize(h, energy_virial), "energy");
    h->last_force_step = step;
    h->have_force_step = true;
    return IRBE_OK;
}

irbe_status irbe_compute_forces_noalloc(irbe_handle h, const void* pos, uint64_t step, void* force, uint32_t flags,
                                        double* energy_virial)
{
    if (!h) return IRBE_EINVAL;
    if (!pos || !force) return fail(h, IRBE_EINVAL, "irbe_compute_forces_noalloc: null argument");
    if (flags & ~(uint32_t)(IRBE_ENERGY | IRBE_VIRIAL)) return fail(h, IRBE_EINVAL, "unknown flags");
    if (flags && !energy_virial) return fail(h, IRBE_EINVAL, "energy/virial requested without a buffer");
    if (!h->have_lists) return fail(h, IRBE_ESTATE, "irbe_compute_forces_noalloc before irbe_build_lists");
    if (h->stencil) return fail(h, IRBE_EUNSUPPORTED, "irbe_compute_forces_noalloc: stencil sampling not supported");
    if (!h->full_list && !draw_bitmaps_in_lds(h))
        return fail(h, IRBE_EUNSUPPORTED,
                    "irbe_compute_forces_noalloc: shell lists longer than the batch draw keeps in LDS");
    hipError_t se = hipSuccess;
    unsigned char* base = (unsigned char*)scratch_addr(h->device, &se);
    if (!base) return hip_fail(h, se, "irbe_compute_forces_noalloc: device address of the scratch array");

    // the per-call buffers of one force evaluation, carved from the scratch array
    const size_t n = (size_t)h->cfg.n_atoms, rs = h->real_size, P = (size_t)h->cfg.p_kspace;
    size_t used = 0;
    auto take = [&](size_t bytes) {
        unsigned char* p = base + used;
        used += (bytes + 255) / 256 * 256;
        return (void*)p;
    };
    void* fsr = take(3 * n * rs);
    double* pair_part = (double*)take((size_t)h->part_blocks * kPairPartials * sizeof(double));
    double* pair_slices = (double*)take(256 * 12 * sizeof(double));
    double* ev_pair = (double*)take(kPairPartials * sizeof(double));
    double* fcorr = (double*)take(3 * sizeof(double));
    int4* kvec = (int4*)take(P * sizeof(int4));
    double* kcoef = (double*)take(4 * P * sizeof(double));
    double* rho_part = (double*)take(2 * P * (size_t)rho_blocks(h->cfg.n_atoms) * sizeof(double));
    double* rho = (double*)take(2 * P * sizeof(double));
    void* kforce = take(P * (h->fp64 ? sizeof(KForce<double>) : sizeof(KForce<float>)));
    uint16_t* ranks = h->p_stride > 0 ? (uint16_t*)take(n * (size_t)h->p_stride * sizeof(uint16_t)) : nullptr;
    if (used > kNoAllocScratchBytes)
        return fail(h, IRBE_ECAPACITY,
                    "irbe_compute_forces_noalloc: this system needs " + std::to_string(used) +
                        " bytes of scratch; the no-allocation scratch holds " + std::to_string(kNoAllocScratchBytes));

    // the launchers take their buffers from the handle: point it at the carved
    // buffers for this call and restore its own afterwards (the kernels already
    // hold the addresses they were given)
    struct Swap {
        irbe_ctx* h;
        void *fsr, *kforce;
        double *pair_part, *pair_slices, *ev_pair, *fcorr, *kcoef, *rho_part, *rho;
        int4* kvec;
        uint16_t* ranks;
        ~Swap()
        {
            h->fsr = fsr;
            h->kforce = kforce;
            h->pair_part = pair_part;
            h->pair_slices = pair_slices;
            h->ev_pair = ev_pair;
            h->fcorr = fcorr;
            h->kcoef = kcoef;
            h->rho_part = rho_part;
            h->rho = rho;
            h->kvec = kvec;
            h->ranks = ranks;
            // the draw of this call lived in the scratch array
            h->ranks_valid = false;
        }
    } saved{h, h->fsr, h->kforce, h->pair_part, h->pair_slices, h->ev_pair, h->fcorr, h->kcoef,
            h->rho_part, h->rho, h->kvec, h->ranks};
    h->fsr = fsr;
    h->kforce = kforce;
    h->pair_part = pair_part;
    h->pair_slices = pair_slices;
    h->ev_pair = ev_pair;
    h->fcorr = fcorr;
    h->kcoef = kcoef;
    h->rho_part = rho_part;
    h->rho = rho;
    h->kvec = kvec;
    h->ranks = ranks;
    h->ranks_valid = false;

    // the launch sequence of irbe_compute_forces, without timing events
    const bool ev = flags != 0;
    IRBE_TRY(h, launch_requantize(h, pos), "quantize");
    IRBE_TRY(h, launch_ksample(h, step), "k sampling");
    IRBE_TRY(h, launch_rho(h, nullptr, false), "structure factor");
    IRBE_TRY(h, launch_pair_forces(h, step, ev), "pair forces");
    IRBE_TRY(h, launch_pair_reduce(h), "pair reduction");
    IRBE_TRY(h, launch_kspace_forces(h, force), "k-space forces");
    if (ev) IRBE_TRY(h, launch_energy_finalize(h, energy_virial), "energy");
    return IRBE_OK;
}

irbe_status irbe_compute_forces_backward(irbe_handle h, const void* pos, uint64_t step, const void* grad_force,
                                         void* grad_pos, void* grad_charge, double* grad_lj)
{
    if (!h) return IRBE_EINVAL;
    if (!pos || !grad_force || !grad_pos) return fail(h, IRBE_EINVAL, "irbe_compute_forces_backward: null argument");
    if (!h->have_lists) return fail(h, IRBE_ESTATE, "backward before irbe_build_lists");
    if (grad_lj && h->cfg.n_types > kMaxTypesGrad)
        return fail(h, IRBE_EUNSUPPORTED, "LJ gradients need n_types <= 4");
    // a backward that follows a forward: the next forward (list-drawn or stencil-
    // drawn batches) also writes the batch atoms, for the backward expected after it
    if (h->fwd_pending && !h->full_list) {
        IRBE_TRY(h, ensure_batch_atoms(h), "allocating the batch atoms");
        h->keep_batch = true;
    }
    h->fwd_pending = false;
    IRBE_STAGE(h, IRBE_STAGE_QUANTIZE, launch_requantize(h, pos), "quantize");
    IRBE_STAGE(h, IRBE_STAGE_KSAMPLE, launch_ksample(h, step), "k sampling");
    IRBE_STAGE(h, IRBE_STAGE_GRAD_GATHER, launch_gather_grad(h, grad_force), "gather dL/dF");
    IRBE_STAGE(h, IRBE_STAGE_RHO_ADJ, launch_rho(h, grad_force, true), "structure factor (adjoint)");
    IRBE_STAGE(h, IRBE_STAGE_PAIR_ADJ, launch_pair_adjoint(h, step, grad_charge != nullptr, grad_lj != nullptr),
               "pair adjoint");
    IRBE_STAGE(h, IRBE_STAGE_KSPACE_ADJ, launch_kspace_adjoint(h, grad_force, grad_pos, grad_charge, grad_lj),
               "k-space adjoint");
    return IRBE_OK;
}

irbe_status irbe_sync(irbe_handle h)
{
    if (!h) return IRBE_EINVAL;
    IRBE_TRY(h, hipStreamSynchronize(h->stream), "synchronize");
    return check_device_error(h);
}

irbe_status irbe_get_debug(irbe_handle h, int32_t what, void* dst_host, int64_t capacity, int64_t* written)
{
    if (!h) return IRBE_EINVAL;
    if (!written || capacity < 0 || (capacity > 0 && !dst_host)) return fail(h, IRBE_EINVAL, "bad debug buffer");
    IRBE_TRY(h, hipStreamSynchronize(h->stream), "synchronize");
    const int64_t n = h->cfg.n_atoms;
    auto copy_out = [&](const void* src, size_t elem, int64_t count) {
        *written = count;
        const int64_t m = std::min(count, capacity);
        if (m > 0) std::memcpy(dst_host, src, (size_t)m * elem);
    };
    auto d2h = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
    };
    const bool needs_lists = what == IRBE_DBG_CELL_START || what == IRBE_DBG_CELL_ATOMS || what == IRBE_DBG_CORE_OFF ||
                             what == IRBE_DBG_CORE_IDX || what == IRBE_DBG_SHELL_OFF || what == IRBE_DBG_SHELL_IDX ||
                             what == IRBE_DBG_BATCH_OFF || what == IRBE_DBG_BATCH_RANK;
    if (needs_lists && !h->have_lists) return fail(h, IRBE_ESTATE, "no lists built");
    const bool needs_force = what == IRBE_DBG_KVEC || what == IRBE_DBG_RHO || what == IRBE_DBG_FCORR ||
                             what == IRBE_DBG_BATCH_OFF || what == IRBE_DBG_BATCH_RANK;
    if (needs_force && !h->have_force_step) return fail(h, IRBE_ESTATE, "no force evaluation yet");
    switch (what) {
    case IRBE_DBG_CELL_START: {
        std::vector<int32_t> v((size_t)h->geo.n_cells + 1);
        IRBE_TRY(h, d2h(v.data(), h->cell_start, v.size() * 4), "debug");
        std::vector<int64_t> w(v.begin(), v.end());
        copy_out(w.data(), 8, (int64_t)w.size());
        return IRBE_OK;
    }
    case IRBE_DBG_CELL_ATOMS: {
        std::vector<int32_t> v((size_t)n);
        IRBE_TRY(h, d2h(v.data(), h->perm, v.size() * 4), "debug");
        std::vector<int64_t> w(v.begin(), v.end());
        copy_out(w.data(), 8, (int64_t)w.size());
        return IRBE_OK;
    }
    case IRBE_DBG_CORE_OFF:
    case IRBE_DBG_CORE_IDX:
    case IRBE_DBG_SHELL_OFF:
    case IRBE_DBG_SHELL_IDX:
    case IRBE_DBG_BATCH_OFF:
    case IRBE_DBG_BATCH_RANK: {
        if (h->stencil && (what == IRBE_DBG_SHELL_OFF || what == IRBE_DBG_SHELL_IDX))
            return fail(h, IRBE_ESTATE, "no shell list with stencil sampling");
        const bool is_core = what == IRBE_DBG_CORE_OFF || what == IRBE_DBG_CORE_IDX;
        const bool is_batch = what == IRBE_DBG_BATCH_OFF || what == IRBE_DBG_BATCH_RANK;
        const bool want_off = what == IRBE_DBG_CORE_OFF || what == IRBE_DBG_SHELL_OFF || what == IRBE_DBG_BATCH_OFF;
        std::vector<int32_t> perm((size_t)n), rank((size_t)n), cnt((size_t)n);
        IRBE_TRY(h, d2h(perm.data(), h->perm, (size_t)n * 4), "debug");
        IRBE_TRY(h, d2h(rank.data(), h->rank, (size_t)n * 4), "debug");
        IRBE_TRY(h, d2h(cnt.data(), is_core ? h->ncore : h->nshell, (size_t)n * 4), "debug");
        int32_t stride = is_core ? h->cap_core : h->cap_shell;
        std::vector<int32_t> rows;
        std::vector<uint16_t> rk;
        if (is_batch) {
            // the ranks the pair kernel used for the step of the last force evaluation
            if (!h->full_list && !(h->ranks_valid && h->ranks_step == h->last_force_step))
                return fail(h, IRBE_ESTATE, "batch ranks of the last force step are not available");
            if (!h->full_list) {
                rk.resize((size_t)n * h->p_stride);
                IRBE_TRY(h, d2h(rk.data(), h->ranks, rk.size() * 2), "debug");
            }
        } else if (!is_core && h->shell16) {
            // 16-bit entries, decoded here
            std::vector<uint16_t> r16((size_t)n * stride);
            std::vector<int32_t> cs((size_t)h->geo.n_cells + 1), grp((size_t)n);
            IRBE_TRY(h, d2h(r16.data(), h->shell, r16.size() * 2), "debug");
            IRBE_TRY(h, d2h(cs.data(), h->cell_start, cs.size() * 4), "debug");
            IRBE_TRY(h, d2h(grp.data(), h->sgroup, grp.size() * 4), "debug");
            rows.assign((size_t)n * stride, 0);
            for (int64_t k = 0; k < n; ++k)
                for (int32_t t = 0; t < cnt[k]; ++t)
                    rows[(size_t)k * stride + t] =
                        decode_shell_entry(h->lcode, cs, grp[k], r16[(size_t)k * stride + t]);
        } else {
            rows.resize((size_t)n * stride);
            IRBE_TRY(h, d2h(rows.data(), is_core ? h->core : h->shell, rows.size() * 4), "debug");
        }
        auto row_len = [&](int64_t k) -> int64_t {
            if (is_core && h->full_list) return 0;
            if (is_batch && !h->full_list) return std::min<int64_t>(cnt[k], h->cfg.p_shell);
            return cnt[k];
        };
        std::vector<int64_t> off((size_t)n + 1, 0);
        for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + row_len(rank[i]);
        if (want_off) {
            copy_out(off.data(), 8, n + 1);
            return IRBE_OK;
        }
        std::vector<int32_t> idx((size_t)off[n]);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t k = rank[i];
            const bool sampled = is_batch && !h->full_list && cnt[k] > h->cfg.p_shell;
            for (int64_t t = 0; t < off[i + 1] - off[i]; ++t) {
                if (is_batch) idx[off[i] + t] = sampled ? (int32_t)rk[(size_t)k * h->p_stride + t] : (int32_t)t;
                else idx[off[i] + t] = perm[rows[(size_t)k * stride + t]];
            }
        }
        copy_out(idx.data(), 4, (int64_t)idx.size());
        return IRBE_OK;
    }
    case IRBE_DBG_KVEC: {
        std::vector<int4> v((size_t)h->cfg.p_kspace);
        IRBE_TRY(h, d2h(v.data(), h->kvec, v.size() * sizeof(int4)), "debug");
        std::vector<int32_t> w;
        for (auto& m : v) {
            w.push_back(m.x);
            w.push_back(m.y);
            w.push_back(m.z);
        }
        copy_out(w.data(), 4, (int64_t)w.size());
        return IRBE_OK;
    }
    case IRBE_DBG_RHO: {
        std::vector<double> v(2 * (size_t)h->cfg.p_kspace);
        IRBE_TRY(h, d2h(v.data(), h->rho, v.size() * 8), "debug");
        copy_out(v.data(), 8, (int64_t)v.size());
        return IRBE_OK;
    }
    case IRBE_DBG_FCORR: {
        double v[3];
        IRBE_TRY(h, d2h(v, h->fcorr, sizeof(v)), "debug");
        copy_out(v, 8, 3);
        return IRBE_OK;
    }
    case IRBE_DBG_COUNTS: {
        if (!h->have_lists) return fail(h, IRBE_ESTATE, "no lists built");
        std::vector<int32_t> a((size_t)n), b((size_t)n);
        IRBE_TRY(h, d2h(a.data(), h->ncore, (size_t)n * 4), "debug");
        IRBE_TRY(h, d2h(b.data(), h->nshell, (size_t)n * 4), "debug");
        int64_t v[4] = {0, 0, h->full_list ? 0 : h->cap_core, h->cap_shell};
        for (int64_t i = 0; i < n; ++i) {
            v[0] += h->full_list ? 0 : a[i];
            v[1] += b[i];
        }
        copy_out(v, 8, 4);
        return IRBE_OK;
    }
    case IRBE_DBG_ADJ_BATCH: {
        const int64_t v = h->adj_used_batch ? 1 : 0;
        copy_out(&v, 8, 1);
        return IRBE_OK;
    }
    case IRBE_DBG_SHELL_BITS: {
        if (!h->have_lists) return fail(h, IRBE_ESTATE, "no lists built");
        const int64_t v = h->shell16 ? 16 : 32;
        copy_out(&v, 8, 1);
        return IRBE_OK;
    }
    case IRBE_DBG_ADJ_ATOMICS: {
        unsigned long long c = 0;
        IRBE_TRY(h, d2h(&c, h->adj_atomics, sizeof(c)), "debug");
        const int64_t v = h->adj_all_atomic ? -1 : (int64_t)c;
        copy_out(&v, 8, 1);
        return IRBE_OK;
    }
    case IRBE_DBG_SCALARS: {
        const double v[4] = {h->kS, h->kH, (double)h->geo.n_c, (double)h->geo.reach};
        copy_out(v, 8, 4);
        return IRBE_OK;
    }
    default:
        return fail(h, IRBE_EINVAL, "unknown debug selector");
    }
}

irbe_status irbe_get_debug_rows(irbe_handle h, int32_t what, const int64_t* rows_host, int64_t n_rows, void* dst_host,
                                int64_t capacity, int64_t* written)
{
    if (!h) return IRBE_EINVAL;
    if (!written || capacity < 0 || (capacity > 0 && !dst_host) || n_rows < 0 || (n_rows > 0 && !rows_host))
        return fail(h, IRBE_EINVAL, "bad debug buffer");
    const bool is_core = what == IRBE_DBG_CORE_OFF || what == IRBE_DBG_CORE_IDX;
    const bool is_shell = what == IRBE_DBG_SHELL_OFF || what == IRBE_DBG_SHELL_IDX;
    const bool is_atoms = what == IRBE_DBG_BATCH_ATOMS;
    const bool is_batch = what == IRBE_DBG_BATCH_OFF || what == IRBE_DBG_BATCH_RANK || is_atoms;
    if (!is_core && !is_shell && !is_batch) return fail(h, IRBE_EINVAL, "selector is not per atom");
    if (is_shell && h->stencil) return fail(h, IRBE_ESTATE, "no shell list with stencil sampling");
    if (!h->have_lists) return fail(h, IRBE_ESTATE, "no lists built");
    if (is_batch && !h->full_list && !(h->have_force_step && h->ranks_valid && h->ranks_step == h->last_force_step))
        return fail(h, IRBE_ESTATE, "batch ranks of the last force step are not available");
    const int64_t n = h->cfg.n_atoms;
    for (int64_t r = 0; r < n_rows; ++r)
        if (rows_host[r] < 0 || rows_host[r] >= n) return fail(h, IRBE_EINVAL, "row id out of range");
    if (is_atoms && h->stencil) IRBE_TRY(h, launch_stencil_decode(h), "decode the batch");
    IRBE_TRY(h, hipStreamSynchronize(h->stream), "synchronize");
    const bool want_off = what == IRBE_DBG_CORE_OFF || what == IRBE_DBG_SHELL_OFF || what == IRBE_DBG_BATCH_OFF;
    std::vector<int32_t> perm;
    if (!want_off && (!is_batch || is_atoms)) {
        perm.resize((size_t)n);
        IRBE_TRY(h, hipMemcpy(perm.data(), h->perm, (size_t)n * 4, hipMemcpyDeviceToHost), "debug");
    }
    std::vector<int64_t> off((size_t)n_rows + 1, 0);
    std::vector<int32_t> idx;
    // the first len entries of sorted atom k's shell row as sorted indices
    std::vector<int32_t> cs16;  // cell starts of the build, for 16-bit entries
    auto read_shell_row = [&](int32_t k, int64_t len, std::vector<int32_t>& row) -> hipError_t {
        row.resize((size_t)len);
        if (!h->shell16)
            return hipMemcpy(row.data(), h->shell + (int64_t)k * h->cap_shell, (size_t)len * 4, hipMemcpyDeviceToHost);
        std::vector<uint16_t> r16((size_t)len);
        int32_t grp = 0;
        hipError_t e = hipMemcpy(r16.data(), reinterpret_cast<const uint16_t*>(h->shell) + (int64_t)k * h->cap_shell,
                                 (size_t)len * 2, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(&grp, h->sgroup + k, 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess && cs16.empty()) {
            cs16.resize((size_t)h->geo.n_cells + 1);
            e = hipMemcpy(cs16.data(), h->cell_start, cs16.size() * 4, hipMemcpyDeviceToHost);
        }
        if (e != hipSuccess) return e;
        for (int64_t t = 0; t < len; ++t) row[(size_t)t] = decode_shell_entry(h->lcode, cs16, grp, r16[(size_t)t]);
        return hipSuccess;
    };
    for (int64_t r = 0; r < n_rows; ++r) {
        int32_t k = 0, cnt = 0;
        IRBE_TRY(h, hipMemcpy(&k, h->rank + rows_host[r], 4, hipMemcpyDeviceToHost), "debug");
        IRBE_TRY(h, hipMemcpy(&cnt, (is_core ? h->ncore : h->nshell) + k, 4, hipMemcpyDeviceToHost), "debug");
        int64_t len = (is_core && h->full_list) ? 0 : cnt;
        const bool sampled = is_batch && !h->full_list && cnt > h->cfg.p_shell;
        if (is_batch && !h->full_list) len = std::min<int64_t>(cnt, h->cfg.p_shell);
        off[r + 1] = off[r] + len;
        if (want_off || len == 0) continue;
        if (is_atoms && h->stencil) {
            // the decoded atoms of the batch (sorted index, -1 for i and its molecule)
            std::vector<int32_t> bj((size_t)len);
            IRBE_TRY(h, hipMemcpy(bj.data(), h->batch_j + (int64_t)k * h->p_stride, (size_t)len * 4,
                                  hipMemcpyDeviceToHost),
                     "debug");
            for (auto v : bj) idx.push_back(v < 0 ? -1 : perm[v]);
        } else if (is_batch) {
            std::vector<int32_t> rv;
            if (sampled) {
                std::vector<uint16_t> rk((size_t)len);
                IRBE_TRY(h, hipMemcpy(rk.data(), h->ranks + (int64_t)k * h->p_stride, (size_t)len * 2,
                                      hipMemcpyDeviceToHost),
                         "debug");
                for (auto v : rk) rv.push_back((int32_t)v);
            } else {
                for (int64_t t = 0; t < len; ++t) rv.push_back((int32_t)t);
            }
            if (is_atoms) {
                // list sampling: the shell members at the ranks
                std::vector<int32_t> row;
                IRBE_TRY(h, read_shell_row(k, cnt, row), "debug");
                for (auto v : rv) idx.push_back(perm[row[v]]);
            } else {
                for (auto v : rv) idx.push_back(v);
            }
        } else {
            std::vector<int32_t> row((size_t)len);
            if (is_core)
                IRBE_TRY(h, hipMemcpy(row.data(), h->core + (int64_t)k * h->cap_core, (size_t)len * 4,
                                      hipMemcpyDeviceToHost),
                         "debug");
            else
                IRBE_TRY(h, read_shell_row(k, len, row), "debug");
            for (auto v : row) idx.push_back(perm[v]);
        }
    }
    if (want_off) {
        *written = n_rows + 1;
        std::memcpy(dst_host, off.data(), (size_t)std::min<int64_t>(capacity, n_rows + 1) * 8);
    } else {
        *written = (int64_t)idx.size();
        if (capacity > 0) std::memcpy(dst_host, idx.data(), (size_t)std::min<int64_t>(capacity, *written) * 4);
    }
    return IRBE_OK;
}

irbe_status irbe_enable_timing(irbe_handle h, int32_t enable)
{
    if (!h) return IRBE_EINVAL;
    IRBE_TRY(h, hipStreamSynchronize(h->stream), "synchronize");
    drain_timing(h);
    for (int s = 0; s < IRBE_N_STAGES; ++s) {
        h->stage_ms[s] = 0.0;
        h->stage_n[s] = 0;
    }
    h->timing = enable != 0;
    return IRBE_OK;
}

irbe_status irbe_get_timing(irbe_handle h, double* ms_host, int64_t capacity, int64_t* written)
{
    if (!h) return IRBE_EINVAL;
    if (!written || capacity < 0 || (capacity > 0 && !ms_host)) return fail(h, IRBE_EINVAL, "bad timing buffer");
    IRBE_TRY(h, hipStreamSynchronize(h->stream), "synchronize");
    drain_timing(h);
    *written = 2 * IRBE_N_STAGES;
    for (int s = 0; s < IRBE_N_STAGES; ++s) {
        if (2 * s < capacity) ms_host[2 * s] = h->stage_ms[s];
        if (2 * s + 1 < capacity) ms_host[2 * s + 1] = (double)h->stage_n[s];
    }
    return IRBE_OK;
}

const char* irbe_last_error(irbe_handle h)
{
    return h ? h->last_error.c_str() : g_create_error.c_str();
}

irbe_status irbe_destroy(irbe_handle h)
{
    if (!h) return IRBE_EINVAL;
    hipStreamSynchronize(h->stream);
    drain_timing(h);
    for (void* p : h->owned) hipFree(p);
    h->owned.clear();
    if (h->chk_host) hipHostFree(h->chk_host);
    if (h->chk_event) hipEventDestroy(h->chk_event);
    delete h;
    return IRBE_OK;
}

}  // extern "C"
