// Host layer of libfasttracks: argument validation, device buffers, tiling
// decisions and the stream-ordered launch sequence behind the C ABI of
// include/fasttracks.h.  No arithmetic of the statistic happens here; the host
// only derives launch parameters (window widths, guard margins) from bounds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <array>
#include <map>
#include <string>
#include <numeric>
#include <random>
#include <utility>
#include <vector>

#include "ft_internal.h"

using namespace ft;

struct ft_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    // SFT set
    bool have_sfts = false, have_vel = false;
    int32_t n_sft = 0, n_bins = 0;
    int64_t first_bin = 0;
    double t_sft = 0.0;
    bool has_weight = false;
    std::vector<double> t_mid_h;
    std::vector<double> v_h;
    double vmax = 0.0;
    double *d_arms = nullptr;
    size_t cap_arms = 0;
    bool have_arms = false;  // d_arms holds the arms of the current SFT set
    float *d_ind = nullptr, *d_ind_w = nullptr;  // number-count tables 1[P > 3.2], u_k 1[P > 3.2]
    size_t cap_ind = 0, cap_ind_w = 0;
    bool ind_valid = false;
    double *d_mu_sigma_nc = nullptr;  // noise moments of the number count
    size_t cap_mu_sigma_nc = 0;
    double *d_sky_norm = nullptr, *d_sky_ms = nullptr;  // sky-dependent weights of the last evaluation
    size_t cap_sky_norm = 0, cap_sky_ms = 0;
    double *d_top_nc = nullptr;  // ft_toplist_number_count staging
    size_t cap_top_nc = 0;
    // binary-track estimate: measured error of the hardware cosine (-1: not yet
    // measured) and the mode (0 auto, 1 library polynomial)
    double hw_cos_err = -1.0;
    int32_t cos_mode = 0;
    unsigned long long *d_cos_err = nullptr;
    size_t cap_cos_err = 0;
    // hyperbox search (ft_eval_binary_boxes)
    int32_t *d_box = nullptr, *d_bcount = nullptr;
    uint32_t *d_bmax32 = nullptr, *d_bncand = nullptr;
    unsigned long long *d_bmax64 = nullptr, *d_bidx = nullptr;
    int64_t *d_bcand = nullptr;
    double *d_bcand_s64 = nullptr;
    ft_box_result *d_bout = nullptr;
    size_t cap_box = 0, cap_bcount = 0, cap_bmax32 = 0, cap_bncand = 0, cap_bmax64 = 0, cap_bidx = 0, cap_bcand = 0,
           cap_bcand_s64 = 0, cap_bout = 0;
    int32_t *d_inj_bin = nullptr;
    size_t cap_inj_bin = 0;
    double *d_inj_amp = nullptr;
    size_t cap_inj_amp = 0;
    GenRun *d_genruns = nullptr;
    size_t cap_genruns = 0;
    int64_t *d_prefix = nullptr;  // generator prefix sums (sft, elements)
    size_t cap_prefix = 0;
    std::vector<GenRun> genruns_h;
    std::vector<int64_t> prefix_h;
    float *d_power = nullptr;
    size_t cap_power = 0;
    float *d_weight = nullptr;
    size_t cap_weight = 0;
    float *d_power_w = nullptr;
    size_t cap_power_w = 0;
    double *d_tmid = nullptr, *d_v = nullptr, *d_dt = nullptr;
    float *d_v32 = nullptr;  // velocities rounded to float (estimates of binary tracks)
    size_t cap_v32 = 0;
    std::vector<float> v32_h;
    size_t cap_tmid = 0, cap_v = 0, cap_dt = 0;
    double *d_mu_sigma = nullptr;
    uint32_t *d_err = nullptr;

    // bank
    std::vector<double> f0_h, f1_h, sky_h, sky_tile_h, ap_h, omega_h, phib_h;
    std::vector<int32_t> perm_h;
    // the grid sky whose Doppler-coherent order sky_tile_h/perm_h and
    // d_sky_tile/d_perm hold (reused while a call brings the same sky, byte for byte)
    std::vector<double> sky_order_of;
    bool sky_order_valid = false;
    double *d_f0 = nullptr, *d_f1 = nullptr, *d_sky = nullptr, *d_edges = nullptr,
           *d_sky_tile = nullptr, *d_bin = nullptr;  // d_bin: binary banks' [3][n] a_p, Omega, phi_b
    size_t cap_f0 = 0, cap_f1 = 0, cap_sky = 0, cap_edges = 0, cap_sky_tile = 0, cap_bin = 0;
    double *d_sincos = nullptr;  // ft_lib_sincos staging
    size_t cap_sincos = 0;
    double *d_genbank = nullptr;  // ft_gen_binary_bank staging: f0 | sky | ap | omega | phib
    size_t cap_genbank = 0;
    double *d_qsample = nullptr;  // ft_q_sample staging
    size_t cap_qsample = 0;
    int32_t *d_perm = nullptr;
    size_t cap_perm = 0;
    double *d_tune_sky = nullptr;  // the autotuner's sky sample (Doppler order) and its
    int32_t *d_tune_perm = nullptr;  // original indices
    size_t cap_tune_sky = 0, cap_tune_perm = 0;
    float *d_stats = nullptr;
    size_t cap_stats = 0;
    float *d_bsum = nullptr;  // block sums of the split binary evaluation
    size_t cap_bsum = 0;

    // selection
    uint32_t *d_hist = nullptr, *d_state = nullptr, *d_cnt = nullptr, *d_off = nullptr,
             *d_fill = nullptr;
    size_t cap_hist = 0, cap_state = 0, cap_cnt = 0, cap_off = 0, cap_fill = 0;
    int64_t *d_cand = nullptr;
    double *d_cand_s64 = nullptr, *d_cand_mom = nullptr;
    size_t cap_cand = 0, cap_cand_s64 = 0, cap_cand_mom = 0;
    int32_t *d_seg = nullptr;
    size_t cap_seg = 0;
    ft_candidate *d_out = nullptr;
    size_t cap_out = 0;
    int32_t *d_nout = nullptr;
    size_t cap_nout = 0;
    unsigned long long *d_count = nullptr;
    int32_t *d_bins = nullptr;
    size_t cap_bins = 0;

    // batches
    struct BatchBufs {
        double *tmid = nullptr, *v = nullptr, *arms = nullptr, *dt = nullptr, *f0 = nullptr, *f1 = nullptr,
               *sky = nullptr, *sky_tile = nullptr, *tref = nullptr, *s64 = nullptr, *maxz = nullptr,
               *inj_amp = nullptr;
        size_t c_tmid = 0, c_v = 0, c_arms = 0, c_dt = 0, c_f0 = 0, c_f1 = 0, c_sky = 0, c_sky_tile = 0,
               c_tref = 0, c_s64 = 0, c_maxz = 0, c_inj_amp = 0;
        float *power = nullptr, *stats = nullptr;
        size_t c_power = 0, c_stats = 0;
        int32_t *perm = nullptr, *sft_begin = nullptr, *nout = nullptr, *inj_bin = nullptr, *band = nullptr;
        size_t c_perm = 0, c_sft_begin = 0, c_nout = 0, c_inj_bin = 0, c_band = 0;
        int64_t *dt_prefix = nullptr, *cand = nullptr, *gen_prefix = nullptr;
        size_t c_dt_prefix = 0, c_cand = 0, c_gen_prefix = 0;
        EvalRun *runs = nullptr;
        size_t c_runs = 0;
        GenRun *gen = nullptr;
        size_t c_gen = 0;
        int2 *items = nullptr;
        size_t c_items = 0;
        unsigned *counters = nullptr;
        size_t c_counters = 0;
        ft_candidate *out = nullptr;
        size_t c_out = 0;
        uint8_t *labels = nullptr;
        size_t c_labels = 0;
    } bb;
    bool have_batch = false;
    int batch_runs = 0, batch_k = 0, batch_cap = 0;
    hipStream_t capture_stream = nullptr;
    // side streams (default priority) and events of a batch's concurrent
    // evaluation launches
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {nullptr, nullptr, nullptr};
    hipEvent_t fork_ev = nullptr, join_ev[kSide] = {nullptr, nullptr, nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipEvent_t bev[2] = {nullptr, nullptr};
    double batch_ms = 0.0;

    // last evaluation
    bool have_eval = false;
    EvalRun last_run{};
    bool last_grid = true;
    int last_k = 0, last_nsub = 0;
    int64_t last_cap = 0;
    double last_rel_err = 0.0;
    int last_tile = -1;
    int last_stat = FT_STAT_POWER;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};

    float *d_probe = nullptr;  // output of the LDS gather probe
    size_t cap_probe = 0;

    // autotuner: shape class -> tile id (0-based), and the last tuning's timings
    std::map<std::vector<int64_t>, int> tune_cache;
    std::vector<ft_tune_entry> tune_log;
    double tune_ms = 0.0;
};

namespace {

ft_status fail(ft_ctx c, ft_status st, const char *fmt, ...)
{
    if (c) {
        char buf[1024];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return st;
}

ft_status hip_fail(ft_ctx c, hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory) return fail(c, FT_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(c, FT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Test hook: FT_FAULT=alloc:n makes the n-th device allocation (1-based) of the
// process fail, to exercise the FT_E_NOMEM path from the host.
int fault_alloc_countdown()
{
    static int n = [] {
        const char *s = getenv("FT_FAULT");
        if (s && strncmp(s, "alloc:", 6) == 0) return atoi(s + 6);
        return 0;
    }();
    return n;
}
int g_alloc_calls = 0;

template <typename T>
hipError_t ensure(T **p, size_t *cap, size_t count)
{
    if (count == 0) count = 1;
    if (*p && *cap >= count) return hipSuccess;
    ++g_alloc_calls;
    if (fault_alloc_countdown() > 0 && g_alloc_calls == fault_alloc_countdown())
        return hipErrorOutOfMemory;
    if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
        *cap = 0;
    }
    const size_t want = std::max(count, *cap + *cap / 4);
    hipError_t e = hipMalloc((void **)p, want * sizeof(T));
    if (e != hipSuccess) {
        e = hipMalloc((void **)p, count * sizeof(T));
        if (e != hipSuccess) {
            *p = nullptr;
            (void)hipGetLastError();
            return hipErrorOutOfMemory;
        }
        *cap = count;
        return hipSuccess;
    }
    *cap = want;
    return hipSuccess;
}

template <typename T>
void release(T **p, size_t *cap)
{
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (cap) *cap = 0;
}

// Copy `count` elements from a host or device pointer into a host vector.
template <typename T>
hipError_t fetch(std::vector<T> &dst, const T *src, size_t count)
{
    dst.resize(count);
    if (count == 0) return hipSuccess;
    return hipMemcpy(dst.data(), src, count * sizeof(T), hipMemcpyDefault);
}

bool is_finite(double x) { return std::isfinite(x); }

ft_status sync_and_check(ft_ctx c)
{
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "stream synchronize");
    uint32_t flags = 0;
    e = hipMemcpy(&flags, c->d_err, sizeof flags, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "read error flags");
    if (flags & ERR_RANGE)
        return fail(c, FT_E_RANGE, "a template track left the SFT table [first_bin, first_bin + n_bins)");
    if (flags & ERR_WINDOW)
        return fail(c, FT_E_INTERNAL, "a tile needed a wider LDS window than the bound allowed");
    if (flags & ERR_BAD_POWER)
        return fail(c, FT_E_INVALID, "power table or weights hold a non-finite or negative value");
    return FT_OK;
}

// Doppler-coherent visiting order of the sky points: bands of equal height in
// sin(declination), right ascension ascending in even bands and descending in
// odd ones, about as many bands as points per band.  Consecutive points are
// then close on the sphere, so the Doppler factors of a tile's sky points
// differ little and its LDS window stays narrow.
void sky_order(const std::vector<double> &sky, int64_t n, std::vector<int32_t> &perm)
{
    perm.resize((size_t)n);
    const int64_t nb = std::max<int64_t>(1, (int64_t)std::llround(std::sqrt((double)n / 3.14159265358979)));
    std::vector<std::pair<double, int32_t>> key((size_t)n);
    for (int64_t s = 0; s < n; ++s) {
        const double x = sky[3 * s], y = sky[3 * s + 1], z = sky[3 * s + 2];
        int64_t band = (int64_t)std::floor((z + 1.0) * 0.5 * (double)nb);
        band = std::min<int64_t>(std::max<int64_t>(band, 0), nb - 1);
        double ra = std::atan2(y, x);
        if (band & 1) ra = -ra;
        key[(size_t)s] = {(double)band * 16.0 + ra, (int32_t)s};
    }
    std::sort(key.begin(), key.end());
    for (int64_t s = 0; s < n; ++s) perm[(size_t)s] = key[(size_t)s].second;
}

// Cost model of a tile: lanes issued per useful template (partial f0 and f1
// tiles) times the VALU operations per evaluation of its inner loop.
double model_cost(int id, double n_f0, double n_f1)
{
    const TileCfg &t = tile_cfg(id);
    const double f0w = std::ceil(n_f0 / (64.0 * t.L)) * 64.0 * t.L / n_f0;
    const double f1w = std::ceil(n_f1 / t.JT) * t.JT / n_f1;
    const double ops = t.L > 1 ? (7.0 + t.L) / t.L : 7.0;
    return f0w * f1w * ops;
}

int choose_tile(int64_t n_f0, int64_t n_f1, bool uniform)
{
    if (!uniform || n_f0 < 96) return n_f1 >= 4 ? 1 : 0;
    // fewest wasted lanes x operations; on ties the first listed (SFT stages
    // of 8 before 16: more workgroups fit in LDS)
    const int cands[] = {8, 3, 2, 4, 5, 7, 6};
    double best = 1e30;
    int best_id = 8;
    for (int id : cands) {
        const double cost = model_cost(id, (double)n_f0, (double)n_f1);
        if (cost < best - 1e-9) {
            best = cost;
            best_id = id;
        }
    }
    return best_id;
}

// Tiles the autotuner times: eligible (run-length tiles need the guard), cost
// model within 1.6x of the best, cheapest first.
std::vector<int> tune_candidates(double n_f0, double n_f1, bool uniform)
{
    std::vector<std::pair<double, int>> cost;
    for (int id = 0; id < tile_count(); ++id)
        if (tile_cfg(id).L == 1 || uniform) cost.push_back({model_cost(id, n_f0, n_f1), id});
    std::stable_sort(cost.begin(), cost.end(),
                     [](const std::pair<double, int> &a, const std::pair<double, int> &b) { return a.first < b.first; });
    std::vector<int> out;
    for (auto &pc : cost)
        if (pc.first <= 1.6 * cost.front().first) out.push_back(pc.second);
    return out;
}

int floor_log2(int64_t x)
{
    int l = 0;
    while (x > 1) {
        x >>= 1;
        ++l;
    }
    return l;
}

}  // namespace

extern "C" {

const char *ft_status_string(int st)
{
    switch (st) {
    case FT_OK: return "FT_OK";
    case FT_E_INVALID: return "FT_E_INVALID";
    case FT_E_STATE: return "FT_E_STATE";
    case FT_E_RANGE: return "FT_E_RANGE";
    case FT_E_NOMEM: return "FT_E_NOMEM";
    case FT_E_DEVICE: return "FT_E_DEVICE";
    case FT_E_UNSUPPORTED: return "FT_E_UNSUPPORTED";
    case FT_E_INTERNAL: return "FT_E_INTERNAL";
    default: return "FT_E_UNKNOWN";
    }
}

int32_t ft_tile_count(void) { return tile_count(); }

// Tile ids of the ABI are 1-based (0 = library choice).
const char *ft_tile_name(int32_t tile)
{
    if (tile < 1 || tile > tile_count()) return "";
    return tile_cfg(tile - 1).name;
}

ft_status ft_tune_report(ft_ctx c, ft_tune_entry *out, int32_t cap, int32_t *n_out, double *tune_ms)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (!n_out) return fail(c, FT_E_INVALID, "n_out must be non-null");
    if (cap < 0 || (cap > 0 && !out)) return fail(c, FT_E_INVALID, "out must hold cap >= 0 entries");
    const int32_t n = (int32_t)std::min<size_t>(c->tune_log.size(), (size_t)cap);
    for (int32_t i = 0; i < n; ++i) out[i] = c->tune_log[(size_t)i];
    *n_out = (int32_t)c->tune_log.size();
    if (tune_ms) *tune_ms = c->tune_ms;
    return FT_OK;
}

ft_status ft_probe_lds_gather(ft_ctx c, int32_t tile, int32_t wtp, double *evals_per_s)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (!evals_per_s) return fail(c, FT_E_INVALID, "evals_per_s must be non-null");
    if (tile < 1 || tile > tile_count()) return fail(c, FT_E_INVALID, "unknown tile %d", tile);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    const TileCfg &cfg = tile_cfg(tile - 1);
    const int min_wtp = (64 * cfg.L + 3 * cfg.JT + 8 + 32 + 63) / 64 * 64;
    if (wtp == 0) wtp = min_wtp;
    if (wtp < min_wtp || wtp % 64 != 0 || 2.0 * cfg.KS * wtp * 4.0 + (double)tile_static_lds(tile - 1) > 150.0 * 1024.0)
        return fail(c, FT_E_INVALID, "wtp must be a multiple of 64 in [%d, LDS budget]", min_wtp);
    const int n_blocks = 2048, n_step = 2048;
    const size_t n_out = (size_t)n_blocks * 64 * cfg.NW;
    hipError_t e = ensure(&c->d_probe, &c->cap_probe, n_out);
    if (e == hipSuccess) e = launch_lds_probe(cfg, n_blocks, 64, wtp, c->d_probe, c->stream);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(c->ev[0], c->stream);
    if (e == hipSuccess) e = launch_lds_probe(cfg, n_blocks, n_step, wtp, c->d_probe, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev[1], c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(c->ev[1]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
    if (e != hipSuccess) return hip_fail(c, e, "LDS gather probe");
    const double evals = (double)n_out * n_step * cfg.JT * cfg.L;
    *evals_per_s = ms > 0.f ? evals / (ms * 1e-3) : 0.0;
    return FT_OK;
}

ft_status ft_probe_lds_read(ft_ctx c, int32_t form, int32_t consume_all, double *bytes_per_s)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (!bytes_per_s) return fail(c, FT_E_INVALID, "bytes_per_s must be non-null");
    if (form < FT_LDS_B32 || form > FT_LDS_READ2ST64_B64) return fail(c, FT_E_INVALID, "unknown LDS read form %d", form);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    const int n_blocks = 8 * 256, n_iter = 4096;
    hipError_t e = ensure(&c->d_probe, &c->cap_probe, (size_t)n_blocks * 256);
    if (e == hipSuccess) e = launch_lds_read_probe(form, consume_all != 0, n_blocks, 64, c->d_probe, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev[0], c->stream);
    if (e == hipSuccess) e = launch_lds_read_probe(form, consume_all != 0, n_blocks, n_iter, c->d_probe, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev[1], c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(c->ev[1]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
    if (e != hipSuccess) return hip_fail(c, e, "LDS read probe");
    const double bytes = (double)n_blocks * 256 * n_iter * 8 * 4.0;
    *bytes_per_s = ms > 0.f ? bytes / (ms * 1e-3) : 0.0;
    return FT_OK;
}

ft_status ft_probe_hbm_read(ft_ctx c, int64_t bytes, double *bytes_per_s)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (!bytes_per_s) return fail(c, FT_E_INVALID, "bytes_per_s must be non-null");
    bytes &= ~(int64_t)15;
    if (bytes < ((int64_t)1 << 30)) return fail(c, FT_E_INVALID, "at least 1 GiB, got %lld", (long long)bytes);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    void *src = nullptr;
    if (hipMalloc(&src, (size_t)bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, FT_E_NOMEM, "HBM probe buffer of %lld bytes", (long long)bytes);
    }
    const int n_blocks = 256 * 16;
    hipError_t e = ensure(&c->d_probe, &c->cap_probe, (size_t)n_blocks * 256);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t *)src, 0u, bytes / 4, c->stream);
    if (e == hipSuccess) e = launch_hbm_read_probe(src, bytes, n_blocks, c->d_probe, c->stream);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(c->ev[0], c->stream);
    const int reps = 5;
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch_hbm_read_probe(src, bytes, n_blocks, c->d_probe, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev[1], c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(c->ev[1]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(src);
    if (e != hipSuccess) return hip_fail(c, e, "HBM read probe");
    *bytes_per_s = ms > 0.f ? (double)bytes * reps / (ms * 1e-3) : 0.0;
    return FT_OK;
}

ft_status ft_tune_clear(ft_ctx c)
{
    if (!c) return FT_E_INVALID;
    c->tune_cache.clear();
    c->tune_log.clear();
    c->tune_ms = 0.0;
    return FT_OK;
}

ft_status ft_create(ft_ctx *out, int device, void *hip_stream)
{
    if (!out) return FT_E_INVALID;
    *out = nullptr;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev <= 0) {
        (void)hipGetLastError();
        return FT_E_DEVICE;
    }
    if (device < 0 || device >= n_dev) return FT_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return FT_E_DEVICE;
    ft_ctx c = new ft_ctx_s();
    c->device = device;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return FT_E_DEVICE;
        }
        c->own_stream = true;
    }
    size_t one = 0;
    if (ensure(&c->d_err, &one, 1) != hipSuccess || hipMalloc(&c->d_mu_sigma, 2 * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->d_count, 2 * sizeof(unsigned long long)) != hipSuccess) {
        ft_destroy(c);
        return FT_E_NOMEM;
    }
    (void)hipMemset(c->d_err, 0, sizeof(uint32_t));
    // the fixed scratch of the no-allocation entry point, resolved once per device
    if (noalloc_scratch_init(device) != hipSuccess) {
        ft_destroy(c);
        return FT_E_DEVICE;
    }
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            ft_destroy(c);
            return FT_E_DEVICE;
        }
    for (auto &e : c->bev)
        if (hipEventCreate(&e) != hipSuccess) {
            ft_destroy(c);
            return FT_E_DEVICE;
        }
    // side streams of a batch's concurrent evaluation launches (created here,
    // outside any graph capture)
    bool side_ok = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < ft_ctx_s::kSide && side_ok; ++i)
        side_ok = hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&c->join_ev[i], hipEventDisableTiming) == hipSuccess;
    if (!side_ok) {
        ft_destroy(c);
        return FT_E_DEVICE;
    }
    *out = c;
    return FT_OK;
}

void ft_destroy(ft_ctx c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    release(&c->d_power, &c->cap_power);
    release(&c->d_weight, &c->cap_weight);
    release(&c->d_power_w, &c->cap_power_w);
    release(&c->d_arms, &c->cap_arms);
    release(&c->d_ind, &c->cap_ind);
    release(&c->d_ind_w, &c->cap_ind_w);
    release(&c->d_mu_sigma_nc, &c->cap_mu_sigma_nc);
    release(&c->d_sky_norm, &c->cap_sky_norm);
    release(&c->d_sky_ms, &c->cap_sky_ms);
    release(&c->d_top_nc, &c->cap_top_nc);
    release(&c->d_cos_err, &c->cap_cos_err);
    release(&c->d_box, &c->cap_box);
    release(&c->d_bcount, &c->cap_bcount);
    release(&c->d_bmax32, &c->cap_bmax32);
    release(&c->d_bncand, &c->cap_bncand);
    release(&c->d_bmax64, &c->cap_bmax64);
    release(&c->d_bidx, &c->cap_bidx);
    release(&c->d_bcand, &c->cap_bcand);
    release(&c->d_bcand_s64, &c->cap_bcand_s64);
    release(&c->d_bout, &c->cap_bout);
    release(&c->d_inj_bin, &c->cap_inj_bin);
    release(&c->d_inj_amp, &c->cap_inj_amp);
    release(&c->d_genruns, &c->cap_genruns);
    release(&c->d_prefix, &c->cap_prefix);
    release(&c->d_tmid, &c->cap_tmid);
    release(&c->d_v, &c->cap_v);
    release(&c->d_v32, &c->cap_v32);
    release(&c->d_dt, &c->cap_dt);
    release(&c->d_mu_sigma, nullptr);
    release(&c->d_err, nullptr);
    release(&c->d_f0, &c->cap_f0);
    release(&c->d_bin, &c->cap_bin);
    release(&c->d_sincos, &c->cap_sincos);
    release(&c->d_genbank, &c->cap_genbank);
    release(&c->d_qsample, &c->cap_qsample);
    release(&c->d_f1, &c->cap_f1);
    release(&c->d_sky, &c->cap_sky);
    release(&c->d_sky_tile, &c->cap_sky_tile);
    release(&c->d_perm, &c->cap_perm);
    release(&c->d_tune_sky, &c->cap_tune_sky);
    release(&c->d_tune_perm, &c->cap_tune_perm);
    release(&c->d_edges, &c->cap_edges);
    release(&c->d_stats, &c->cap_stats);
    release(&c->d_bsum, &c->cap_bsum);
    release(&c->d_hist, &c->cap_hist);
    release(&c->d_state, &c->cap_state);
    release(&c->d_cnt, &c->cap_cnt);
    release(&c->d_off, &c->cap_off);
    release(&c->d_fill, &c->cap_fill);
    release(&c->d_cand, &c->cap_cand);
    release(&c->d_cand_s64, &c->cap_cand_s64);
    release(&c->d_cand_mom, &c->cap_cand_mom);
    release(&c->d_seg, &c->cap_seg);
    release(&c->d_out, &c->cap_out);
    release(&c->d_nout, &c->cap_nout);
    release(&c->d_count, nullptr);
    release(&c->d_bins, &c->cap_bins);
    {
        auto &b = c->bb;
        release(&b.tmid, &b.c_tmid);
        release(&b.v, &b.c_v);
        release(&b.arms, &b.c_arms);
        release(&b.dt, &b.c_dt);
        release(&b.f0, &b.c_f0);
        release(&b.f1, &b.c_f1);
        release(&b.sky, &b.c_sky);
        release(&b.sky_tile, &b.c_sky_tile);
        release(&b.tref, &b.c_tref);
        release(&b.s64, &b.c_s64);
        release(&b.maxz, &b.c_maxz);
        release(&b.inj_amp, &b.c_inj_amp);
        release(&b.power, &b.c_power);
        release(&b.stats, &b.c_stats);
        release(&b.perm, &b.c_perm);
        release(&b.sft_begin, &b.c_sft_begin);
        release(&b.nout, &b.c_nout);
        release(&b.inj_bin, &b.c_inj_bin);
        release(&b.band, &b.c_band);
        release(&b.dt_prefix, &b.c_dt_prefix);
        release(&b.cand, &b.c_cand);
        release(&b.gen_prefix, &b.c_gen_prefix);
        release(&b.runs, &b.c_runs);
        release(&b.gen, &b.c_gen);
        release(&b.items, &b.c_items);
        release(&b.counters, &b.c_counters);
        release(&c->d_probe, &c->cap_probe);
        release(&b.out, &b.c_out);
        release(&b.labels, &b.c_labels);
    }
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    for (int i = 0; i < ft_ctx_s::kSide; ++i) {
        if (c->side[i]) (void)hipStreamDestroy(c->side[i]);
        if (c->join_ev[i]) (void)hipEventDestroy(c->join_ev[i]);
    }
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    for (auto &e : c->bev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *ft_last_error(ft_ctx c) { return c ? c->err.c_str() : "null context"; }

ft_status ft_set_sfts(ft_ctx c, int32_t n_det, const int32_t *n_sft, const double *t_mid,
                      double t_sft, int64_t first_bin, int32_t n_bins, const float *power,
                      const float *weight)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    if (n_det < 1 || !n_sft || !t_mid || !power)
        return fail(c, FT_E_INVALID, "n_det >= 1 and non-null n_sft, t_mid, power are required");
    std::vector<int32_t> counts;
    if (fetch(counts, n_sft, (size_t)n_det) != hipSuccess)
        return fail(c, FT_E_INVALID, "cannot read n_sft");
    int64_t total = 0;
    for (int32_t n : counts) {
        if (n < 1) return fail(c, FT_E_INVALID, "every detector needs at least one SFT");
        total += n;
    }
    if (total > 0x7fffffff) return fail(c, FT_E_UNSUPPORTED, "more than 2^31-1 SFTs");
    if (!(t_sft > 0.0) || !is_finite(t_sft)) return fail(c, FT_E_INVALID, "t_sft must be finite and > 0");
    if (n_bins < 1) return fail(c, FT_E_INVALID, "n_bins must be >= 1");
    if (first_bin < 0 || first_bin + (int64_t)n_bins >= 0x7fffffffLL)
        return fail(c, FT_E_UNSUPPORTED, "bins must lie in [0, 2^31-1)");
    std::vector<double> tm;
    if (fetch(tm, t_mid, (size_t)total) != hipSuccess) return fail(c, FT_E_INVALID, "cannot read t_mid");
    for (double t : tm)
        if (!is_finite(t)) return fail(c, FT_E_INVALID, "t_mid holds a non-finite value");
    hipError_t e;
    const size_t n_cells = (size_t)total * (size_t)n_bins;
    if ((e = ensure(&c->d_power, &c->cap_power, n_cells)) != hipSuccess) return hip_fail(c, e, "alloc power");
    if ((e = ensure(&c->d_tmid, &c->cap_tmid, (size_t)total)) != hipSuccess) return hip_fail(c, e, "alloc t_mid");
    if ((e = ensure(&c->d_dt, &c->cap_dt, (size_t)total)) != hipSuccess) return hip_fail(c, e, "alloc dt");
    if (weight && ((e = ensure(&c->d_weight, &c->cap_weight, (size_t)total)) != hipSuccess ||
                   (e = ensure(&c->d_power_w, &c->cap_power_w, n_cells)) != hipSuccess))
        return hip_fail(c, e, "alloc weight");
    e = hipMemcpyAsync(c->d_power, power, n_cells * sizeof(float), hipMemcpyDefault, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_tmid, tm.data(), (size_t)total * sizeof(double), hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess && weight)
        e = hipMemcpyAsync(c->d_weight, weight, (size_t)total * sizeof(float), hipMemcpyDefault, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy SFT data");
    // Validate the table on the device (it may be large and device-resident).
    if ((e = launch_fill_u32(c->d_err, 0u, 1, c->stream)) != hipSuccess) return hip_fail(c, e, "clear flags");
    if ((e = launch_check_table(c->d_power, weight ? c->d_weight : nullptr, total, n_bins, c->d_err,
                                c->stream)) != hipSuccess)
        return hip_fail(c, e, "check table");
    if ((e = launch_noise_moments(weight ? c->d_weight : nullptr, (int)total, FT_STAT_POWER, c->d_mu_sigma,
                                  c->stream)) != hipSuccess)
        return hip_fail(c, e, "noise moments");
    // The grid kernel stages w_k * P[k][b] (FP32 product) directly into LDS.
    if (weight && (e = launch_weight_table(c->d_power, c->d_weight, c->d_power_w, total, n_bins,
                                           c->stream)) != hipSuccess)
        return hip_fail(c, e, "weight table");
    ft_status st = sync_and_check(c);
    if (st != FT_OK) {
        c->have_sfts = false;
        launch_fill_u32(c->d_err, 0u, 1, c->stream);
        return st;
    }
    if (c->have_sfts && c->n_sft != (int32_t)total) c->have_vel = c->have_arms = false;
    c->ind_valid = false;
    c->n_sft = (int32_t)total;
    c->n_bins = n_bins;
    c->first_bin = first_bin;
    c->t_sft = t_sft;
    c->has_weight = weight != nullptr;
    c->t_mid_h.swap(tm);
    c->have_sfts = true;
    c->have_eval = false;
    return FT_OK;
}

static ft_status set_velocities_impl(ft_ctx c, const double *v, bool sync);

ft_status ft_set_velocities(ft_ctx c, const double *v) { return set_velocities_impl(c, v, true); }

ft_status ft_set_arms(ft_ctx c, const double *arms)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    if (!c->have_sfts) return fail(c, FT_E_STATE, "ft_set_sfts must come first");
    if (!arms) return fail(c, FT_E_INVALID, "arms is null");
    std::vector<double> ah;
    if (fetch(ah, arms, (size_t)c->n_sft * 6) != hipSuccess) return fail(c, FT_E_INVALID, "cannot read arms");
    for (size_t q = 0; q < ah.size(); q += 3) {
        const double n2 = ah[q] * ah[q] + ah[q + 1] * ah[q + 1] + ah[q + 2] * ah[q + 2];
        if (!is_finite(n2) || std::fabs(std::sqrt(n2) - 1.0) > 1e-6)
            return fail(c, FT_E_INVALID, "arm vector %zu (SFT %zu) is not a unit vector", q / 3 % 2, q / 6);
    }
    hipError_t e = ensure(&c->d_arms, &c->cap_arms, ah.size());
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_arms, ah.data(), ah.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "upload arms");
    c->have_arms = true;
    return FT_OK;
}

// Number-count tables of the current SFT set (built on first use).
static ft_status ensure_nc(ft_ctx c)
{
    if (c->ind_valid) return FT_OK;
    const size_t n_cells = (size_t)c->n_sft * (size_t)c->n_bins;
    hipError_t e;
    if ((e = ensure(&c->d_ind, &c->cap_ind, n_cells)) != hipSuccess ||
        (c->has_weight && (e = ensure(&c->d_ind_w, &c->cap_ind_w, n_cells)) != hipSuccess) ||
        (e = ensure(&c->d_mu_sigma_nc, &c->cap_mu_sigma_nc, 2)) != hipSuccess)
        return hip_fail(c, e, "alloc number-count tables");
    e = launch_nc_table(c->d_power, c->has_weight ? c->d_weight : nullptr, c->d_ind, c->d_ind_w, c->n_sft, c->n_bins,
                        c->stream);
    if (e == hipSuccess)
        e = launch_noise_moments(c->has_weight ? c->d_weight : nullptr, c->n_sft, FT_STAT_NUMBER_COUNT,
                                 c->d_mu_sigma_nc, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "number-count tables");
    c->ind_valid = true;
    return FT_OK;
}

static ft_status set_velocities_impl(ft_ctx c, const double *v, bool sync)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (!c->have_sfts) return fail(c, FT_E_STATE, "ft_set_sfts must come first");
    if (!v) return fail(c, FT_E_INVALID, "v_over_c is null");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    std::vector<double> vh;
    const size_t n3 = (size_t)c->n_sft * 3;
    if (fetch(vh, v, n3) != hipSuccess) return fail(c, FT_E_INVALID, "cannot read v_over_c");
    double vmax = 0.0;
    for (size_t k = 0; k < (size_t)c->n_sft; ++k) {
        const double x = vh[3 * k], y = vh[3 * k + 1], z = vh[3 * k + 2];
        if (!is_finite(x) || !is_finite(y) || !is_finite(z)) return fail(c, FT_E_INVALID, "v_over_c holds a non-finite value");
        const double m = std::sqrt(x * x + y * y + z * z);
        if (!(m < 1.0)) return fail(c, FT_E_INVALID, "|v|/c must be < 1 (SFT %zu)", k);
        vmax = std::max(vmax, m);
    }
    hipError_t e = ensure(&c->d_v, &c->cap_v, n3);
    if (e == hipSuccess) e = ensure(&c->d_v32, &c->cap_v32, n3);
    if (e != hipSuccess) return hip_fail(c, e, "alloc velocities");
    c->v32_h.resize(n3);
    for (size_t q = 0; q < n3; ++q) c->v32_h[q] = (float)vh[q];
    e = hipMemcpyAsync(c->d_v, vh.data(), n3 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_v32, c->v32_h.data(), n3 * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && sync) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy velocities");
    c->v_h.swap(vh);
    c->vmax = vmax;
    c->have_vel = true;
    c->have_eval = false;
    return FT_OK;
}

// Validation of one injected signal; returns an error text or nullptr.
static const char *injection_error(const ft_injection &in)
{
    const double vals[] = {in.amp, in.cos_iota, in.psi, in.sky[0], in.sky[1], in.sky[2], in.f0, in.f1,
                           in.ap, in.omega, in.phib};
    for (double x : vals)
        if (!std::isfinite(x)) return "injection parameters must be finite";
    if (in.amp < 0.0 || in.cos_iota < -1.0 || in.cos_iota > 1.0) return "injection needs amp >= 0 and cos_iota in [-1, 1]";
    if (in.amp > 0.0 && std::fabs(std::sqrt(in.sky[0] * in.sky[0] + in.sky[1] * in.sky[1] + in.sky[2] * in.sky[2]) - 1.0) > 1e-12)
        return "injection sky must be a unit vector";
    if (in.amp > 0.0 && !(in.f0 > 0.0)) return "injection f0 must be > 0";
    if (in.ap < 0.0 || in.omega < 0.0) return "injection needs ap >= 0 and omega >= 0";
    if (in.ap > 0.0 && !(in.ap * in.omega < 0.5)) return "injection needs ap * omega < 1/2";
    if (in.ap > 0.0 && !(std::fabs(in.phib) < 1e6)) return "injection phib must satisfy |phib| < 1e6";
    return nullptr;
}

ft_status ft_gen_sfts(ft_ctx c, int32_t n_det, const int32_t *n_sft, const double *t_mid, double t_sft,
                      int64_t first_bin, int32_t n_bins, const double *v_over_c, const double *arms,
                      uint64_t seed, uint32_t run, double t_ref, const ft_injection *inj, int32_t n_inj,
                      float *power_out)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    if (n_det < 1 || !n_sft || !t_mid || !v_over_c || !arms)
        return fail(c, FT_E_INVALID, "n_det >= 1 and non-null n_sft, t_mid, v_over_c, arms are required");
    std::vector<int32_t> counts;
    if (fetch(counts, n_sft, (size_t)n_det) != hipSuccess) return fail(c, FT_E_INVALID, "cannot read n_sft");
    int64_t total = 0;
    for (int32_t n : counts) {
        if (n < 1) return fail(c, FT_E_INVALID, "every detector needs at least one SFT");
        total += n;
    }
    if (total > 0x7fffffff) return fail(c, FT_E_UNSUPPORTED, "more than 2^31-1 SFTs");
    if (!(t_sft > 0.0) || !is_finite(t_sft) || !is_finite(t_ref))
        return fail(c, FT_E_INVALID, "t_sft must be finite and > 0, t_ref finite");
    if (n_bins < 1) return fail(c, FT_E_INVALID, "n_bins must be >= 1");
    if (first_bin < 0 || first_bin + (int64_t)n_bins >= 0x7fffffffLL)
        return fail(c, FT_E_UNSUPPORTED, "bins must lie in [0, 2^31-1)");
    if (n_inj < 0 || n_inj > 64 || (n_inj > 0 && !inj))
        return fail(c, FT_E_INVALID, "n_inj must be in [0, 64] with inj holding n_inj signals");
    std::vector<ft_injection> ins;
    if (n_inj > 0 && fetch(ins, inj, (size_t)n_inj) != hipSuccess) return fail(c, FT_E_INVALID, "cannot read inj");
    for (const ft_injection &in : ins) {
        const char *msg = injection_error(in);
        if (msg) return fail(c, FT_E_INVALID, "%s", msg);
    }
    std::vector<double> tm, ah;
    if (fetch(tm, t_mid, (size_t)total) != hipSuccess || fetch(ah, arms, (size_t)total * 6) != hipSuccess)
        return fail(c, FT_E_INVALID, "cannot read t_mid / arms");
    for (double t : tm)
        if (!is_finite(t)) return fail(c, FT_E_INVALID, "t_mid holds a non-finite value");
    for (double a : ah)
        if (!is_finite(a)) return fail(c, FT_E_INVALID, "arms hold a non-finite value");
    // SFT bookkeeping first (as ft_set_sfts), then the velocities
    hipError_t e;
    const size_t n_cells = (size_t)total * (size_t)n_bins;
    if ((e = ensure(&c->d_power, &c->cap_power, n_cells)) != hipSuccess ||
        (e = ensure(&c->d_tmid, &c->cap_tmid, (size_t)total)) != hipSuccess ||
        (e = ensure(&c->d_dt, &c->cap_dt, (size_t)total)) != hipSuccess ||
        (e = ensure(&c->d_arms, &c->cap_arms, (size_t)total * 6)) != hipSuccess ||
        (e = ensure(&c->d_inj_bin, &c->cap_inj_bin, (size_t)total * std::max(n_inj, 1))) != hipSuccess ||
        (e = ensure(&c->d_inj_amp, &c->cap_inj_amp, (size_t)total * 3 * std::max(n_inj, 1))) != hipSuccess)
        return hip_fail(c, e, "alloc generated SFTs");
    e = hipMemcpyAsync(c->d_tmid, tm.data(), (size_t)total * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_arms, ah.data(), ah.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy SFT times");
    c->have_sfts = true;
    c->n_sft = (int32_t)total;
    c->n_bins = n_bins;
    c->first_bin = first_bin;
    c->t_sft = t_sft;
    c->has_weight = false;
    c->t_mid_h.swap(tm);
    c->have_eval = false;
    c->have_vel = false;
    c->have_arms = true;
    c->ind_valid = false;
    ft_status st = set_velocities_impl(c, v_over_c, false);
    if (st != FT_OK) {
        c->have_sfts = false;
        return st;
    }
    // records 0..n_inj-1 prepare one signal each; record n_inj is the table
    GenRun g{};
    g.seed = seed;
    g.run = run;
    g.sft_offset = 0;
    g.n_sft = (int32_t)total;
    g.n_bins = n_bins;
    g.first_bin = first_bin;
    g.t_mid = c->d_tmid;
    g.v = c->d_v;
    g.arms = c->d_arms;
    g.t_ref = t_ref;
    g.t_sft = t_sft;
    g.table = c->d_power;
    c->genruns_h.clear();
    c->prefix_h.clear();
    for (int i = 0; i < n_inj; ++i) {
        GenRun p = g;
        const ft_injection &in = ins[(size_t)i];
        p.amp = in.amp;
        p.cos_iota = in.cos_iota;
        p.psi = in.psi;
        for (int d = 0; d < 3; ++d) p.sky[d] = in.sky[d];
        p.f0 = in.f0;
        p.f1 = in.f1;
        p.ap = in.ap;
        p.omega = in.omega;
        p.phib = in.phib;
        p.inj_bin = c->d_inj_bin + (int64_t)i * total;
        p.inj_amp = c->d_inj_amp + 3 * (int64_t)i * total;
        p.n_inj = 1;
        c->genruns_h.push_back(p);
        c->prefix_h.push_back((int64_t)i * total);
    }
    c->prefix_h.push_back((int64_t)n_inj * total);
    g.inj_bin = c->d_inj_bin;
    g.inj_amp = c->d_inj_amp;
    g.n_inj = n_inj;
    c->genruns_h.push_back(g);
    c->prefix_h.push_back(0);
    c->prefix_h.push_back(total);
    const size_t n_rec = c->genruns_h.size(), n_pre = c->prefix_h.size();
    if ((e = ensure(&c->d_genruns, &c->cap_genruns, n_rec)) != hipSuccess ||
        (e = ensure(&c->d_prefix, &c->cap_prefix, n_pre)) != hipSuccess)
        return hip_fail(c, e, "alloc generator descriptors");
    e = hipMemcpyAsync(c->d_genruns, c->genruns_h.data(), n_rec * sizeof(GenRun), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_prefix, c->prefix_h.data(), n_pre * sizeof(int64_t), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = launch_gen_tables(c->d_genruns, n_inj, c->d_prefix, (int64_t)n_inj * total, c->d_genruns + n_inj, 1,
                              c->d_prefix + (n_inj + 1), total, c->stream);
    if (e == hipSuccess) e = launch_noise_moments(nullptr, (int)total, FT_STAT_POWER, c->d_mu_sigma, c->stream);
    if (e == hipSuccess && power_out)
        e = hipMemcpyAsync(power_out, c->d_power, n_cells * sizeof(float), hipMemcpyDefault, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->have_sfts = false;
        return hip_fail(c, e, "generate table");
    }
    return FT_OK;
}

// Guard parameters of a uniform f0 grid: dT = spacing * T_sft and eta, the
// bound (in bins) on the rounding of the canonical x + 1/2 and of the estimate
// (f0 + c + 1/(2 g T)) * (g T) (each below 6 * 2^-53 * x_max), the grid's
// deviation tau from uniform spacing and the rounding of the per-SFT drift
// e = dT*g - 1 over a run; doubled for margin.
static void guard_params(const double *f0, int64_t n0, double f0_max, double x_max, double vmax,
                         double T, double &dT, double &eta)
{
    dT = n0 > 1 ? (f0[n0 - 1] - f0[0]) / (double)(n0 - 1) * T : T;
    double tau = 0.0;
    for (int64_t i = 0; i < n0; ++i) tau = std::max(tau, std::fabs(f0[i] - f0[0] - (double)i * (dT / T)));
    tau += 8.0 * std::ldexp(f0_max, -52);
    const double rho = 6.0 * std::ldexp(x_max, -53);
    eta = 2.0 * (2.0 * rho + 2.0 * tau * (1.0 + vmax) * T + std::ldexp(1.0, -40));
}

struct WindowPlan {
    int tile = -1;  // -1: direct kernel
    int32_t wt = 0, wtp = 0, tiles_f0 = 0, tiles_f1 = 0, tiles_sky = 0;
};

// LDS window of a tile shape: bound on hi - lo over every tile and SFT.  The
// f0 span of a tile, the spindown spread of its f1 values and the Doppler
// spread of its sky points (|g - g'| <= vmax |n - n'|) bound the exact range.
static WindowPlan plan_window(const double *f0, int64_t n0, const double *f1, int64_t n1,
                              const double *sky_tile, int64_t ns, double dt_absmax, double vmax,
                              double T, int tile)
{
    WindowPlan wp;
    const TileCfg &cfg = tile_cfg(tile);
    double span_f0 = 0.0;
    for (int64_t i0 = 0; i0 < n0; i0 += 64 * cfg.L) {
        const int64_t i1 = std::min<int64_t>(i0 + 64 * cfg.L, n0) - 1;
        span_f0 = std::max(span_f0, f0[i1] - f0[i0]);
    }
    double span_f1 = 0.0, f1_absmax = 0.0;
    for (int64_t j0 = 0; j0 < n1; j0 += cfg.JT) {
        double lo = f1[j0], hi = lo;
        for (int64_t j = j0; j < std::min<int64_t>(j0 + cfg.JT, n1); ++j) {
            lo = std::min(lo, f1[j]);
            hi = std::max(hi, f1[j]);
        }
        span_f1 = std::max(span_f1, hi - lo);
    }
    for (int64_t j = 0; j < n1; ++j) f1_absmax = std::max(f1_absmax, std::fabs(f1[j]));
    double diam = 0.0;
    for (int64_t s0 = 0; s0 < ns; s0 += cfg.NW)
        for (int64_t a = s0; a < std::min<int64_t>(s0 + cfg.NW, ns); ++a)
            for (int64_t b2 = a + 1; b2 < std::min<int64_t>(s0 + cfg.NW, ns); ++b2) {
                const double dx = sky_tile[3 * a] - sky_tile[3 * b2];
                const double dy = sky_tile[3 * a + 1] - sky_tile[3 * b2 + 1];
                const double dz = sky_tile[3 * a + 2] - sky_tile[3 * b2 + 2];
                diam = std::max(diam, std::sqrt(dx * dx + dy * dy + dz * dz));
            }
    const double a_max = f0[n0 - 1] + f1_absmax * dt_absmax;
    const double width = (span_f0 + span_f1 * dt_absmax) * (1.0 + vmax) * T + a_max * vmax * diam * (1.0 + 1e-9) * T;
    const double wt = std::ceil(width * (1.0 + 1e-9)) + 3.0 + cfg.L;
    const double wtp = std::ceil(wt / 64.0) * 64.0;
    if (2.0 * wtp * cfg.KS * 4.0 + (double)tile_static_lds(tile) > 150.0 * 1024.0) return wp;
    wp.tile = tile;
    wp.wt = (int32_t)wt;
    wp.wtp = (int32_t)wtp;
    wp.tiles_f0 = (int32_t)((n0 + 64 * cfg.L - 1) / (64 * cfg.L));
    wp.tiles_f1 = (int32_t)((n1 + cfg.JT - 1) / cfg.JT);
    wp.tiles_sky = (int32_t)((ns + cfg.NW - 1) / cfg.NW);
    return wp;
}

// Largest hardware-cosine error accepted for the binary-track estimate (the
// guard margin grows with it; beyond this the polynomial estimate is used).
constexpr double kHwCosMaxErr = 1e-4;

// The cosine bound of binary runs: measured once per context (every float in
// [0, 1] through v_cos_f32 against the library cosine, a few milliseconds),
// then delta = err + 2.1e-7 (phase roundings); 0 selects the polynomial.
static ft_status binary_cos_delta(ft_ctx c, double &delta)
{
    delta = 0.0;
    if (c->cos_mode == 1) return FT_OK;
    if (c->hw_cos_err < 0.0) {
        hipError_t e = ensure(&c->d_cos_err, &c->cap_cos_err, 1);
        unsigned long long bits = 0;
        if (e == hipSuccess) e = launch_hw_cos_error(c->d_cos_err, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&bits, c->d_cos_err, sizeof bits, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "measure the hardware cosine");
        double err;
        memcpy(&err, &bits, sizeof err);
        c->hw_cos_err = is_finite(err) ? err : 1e300;
    }
    if (c->hw_cos_err <= kHwCosMaxErr) delta = c->hw_cos_err * (1.0 + 1e-3) + 2.1e-7;
    return FT_OK;
}

// Every canonical bin of f0 (1 + v.n - a_p Omega cos) lies within
// f0 (1 -+ (vmax + aw)) T + 1/2 (a bin of margin each side for roundings).
static bool binary_range_ok(ft_ctx c, double f0_lo, double f0_hi, double aw_max)
{
    const double lo = std::floor(f0_lo * (1.0 - c->vmax - aw_max) * c->t_sft + 0.5) - 2.0;
    const double hi = std::floor(f0_hi * (1.0 + c->vmax + aw_max) * c->t_sft + 0.5) + 2.0;
    return lo >= (double)c->first_bin && hi < (double)c->first_bin + (double)c->n_bins;
}

static ft_status prepare_bank(ft_ctx c, const ft_bank *bank, double t_ref, EvalRun &run,
                              bool &grid, int64_t &n_t)
{
    if (!bank) return fail(c, FT_E_INVALID, "bank is null");
    if (!c->have_sfts || !c->have_vel) return fail(c, FT_E_STATE, "ft_set_sfts and ft_set_velocities must come first");
    if (!is_finite(t_ref)) return fail(c, FT_E_INVALID, "t_ref must be finite");
    grid = bank->kind == FT_BANK_GRID;
    const bool binary = bank->kind == FT_BANK_BINARY;
    if (!grid && !binary && bank->kind != FT_BANK_LIST) return fail(c, FT_E_INVALID, "unknown bank kind %d", bank->kind);
    if (!bank->f0 || (!binary && !bank->f1) || !bank->sky_xyz) return fail(c, FT_E_INVALID, "bank arrays must be non-null");
    if (binary && (!bank->ap || !bank->omega || !bank->phib))
        return fail(c, FT_E_INVALID, "binary banks need ap, omega and phib");
    if (binary && c->n_bins >= (1 << 28)) return fail(c, FT_E_UNSUPPORTED, "binary banks need tables of fewer than 2^28 columns");
    int64_t n0, n1, ns;
    if (grid) {
        n0 = bank->n_f0;
        n1 = bank->n_f1;
        ns = bank->n_sky;
        if (n0 < 1 || n1 < 1 || ns < 1) return fail(c, FT_E_INVALID, "grid sizes must be >= 1");
        if (n0 > 0x7fffffff || n1 > 0x7fffffff || ns > 0x7fffffff)
            return fail(c, FT_E_UNSUPPORTED, "grid dimension above 2^31-1");
    } else {
        n0 = n1 = ns = bank->n_list;
        if (n0 < 1) return fail(c, FT_E_INVALID, "n_list must be >= 1");
    }
    n_t = grid ? n0 * n1 * ns : n0;
    if (grid && (n_t / ns / n1 != n0 || n_t > (1LL << 40)))
        return fail(c, FT_E_UNSUPPORTED, "more than 2^40 templates in one call");
    hipError_t e;
    if (fetch(c->f0_h, bank->f0, (size_t)n0) != hipSuccess || fetch(c->sky_h, bank->sky_xyz, (size_t)ns * 3) != hipSuccess)
        return fail(c, FT_E_INVALID, "cannot read the bank arrays");
    if (binary) {
        c->f1_h.assign((size_t)n1, 0.0);  // no spindown in the binary model
        if (fetch(c->ap_h, bank->ap, (size_t)n0) != hipSuccess || fetch(c->omega_h, bank->omega, (size_t)n0) != hipSuccess ||
            fetch(c->phib_h, bank->phib, (size_t)n0) != hipSuccess)
            return fail(c, FT_E_INVALID, "cannot read the binary parameters");
    } else if (fetch(c->f1_h, bank->f1, (size_t)n1) != hipSuccess) {
        return fail(c, FT_E_INVALID, "cannot read the bank arrays");
    }
    // validation
    double dt_min = c->t_mid_h[0] - t_ref, dt_max = dt_min;
    for (double t : c->t_mid_h) {
        dt_min = std::min(dt_min, t - t_ref);
        dt_max = std::max(dt_max, t - t_ref);
    }
    double f0_min = 1e300, f0_max = -1e300, f1_min = 1e300, f1_max = -1e300;
    for (int64_t i = 0; i < n0; ++i) {
        const double f = c->f0_h[i];
        if (!is_finite(f) || !(f > 0.0)) return fail(c, FT_E_INVALID, "f0 must be finite and > 0");
        if (grid && i > 0 && !(f > c->f0_h[i - 1])) return fail(c, FT_E_INVALID, "grid f0 must be strictly increasing");
        f0_min = std::min(f0_min, f);
        f0_max = std::max(f0_max, f);
    }
    for (int64_t j = 0; j < n1; ++j) {
        const double f = c->f1_h[j];
        if (!is_finite(f)) return fail(c, FT_E_INVALID, "f1 must be finite");
        f1_min = std::min(f1_min, f);
        f1_max = std::max(f1_max, f);
    }
    for (int64_t s = 0; s < ns; ++s) {
        const double x = c->sky_h[3 * s], y = c->sky_h[3 * s + 1], z = c->sky_h[3 * s + 2];
        if (!is_finite(x) || !is_finite(y) || !is_finite(z)) return fail(c, FT_E_INVALID, "sky holds a non-finite value");
        if (std::fabs(std::sqrt(x * x + y * y + z * z) - 1.0) > 1e-12)
            return fail(c, FT_E_INVALID, "sky vectors must have unit norm (template %lld)", (long long)s);
    }
    // every f0 + f1*dt must be positive; bins must fit in int32
    double c_min = 0.0, c_max = 0.0;
    {
        const double cs[4] = {f1_min * dt_min, f1_min * dt_max, f1_max * dt_min, f1_max * dt_max};
        c_min = *std::min_element(cs, cs + 4);
        c_max = *std::max_element(cs, cs + 4);
    }
    if (grid) {
        if (!(f0_min + c_min > 0.0)) return fail(c, FT_E_INVALID, "f0 + f1*(t - t_ref) must stay > 0");
    } else {
        for (int64_t t = 0; t < n0; ++t) {
            const double a = c->f0_h[t] + std::min(c->f1_h[t] * dt_min, c->f1_h[t] * dt_max);
            if (!(a > 0.0)) return fail(c, FT_E_INVALID, "f0 + f1*(t - t_ref) must stay > 0 (template %lld)", (long long)t);
        }
    }
    double aw_max = 0.0;
    if (binary) {
        // the orbital phase stays inside the library cosine's reduction range,
        // and the track frequency stays positive: a_p Omega < 1/2
        const double dt_abs = std::max(std::fabs(dt_min), std::fabs(dt_max));
        for (int64_t t = 0; t < n0; ++t) {
            const double ap = c->ap_h[t], om = c->omega_h[t], pb = c->phib_h[t];
            if (!is_finite(ap) || !is_finite(om) || !is_finite(pb) || ap < 0.0 || om < 0.0)
                return fail(c, FT_E_INVALID, "binary parameters must be finite, a_p >= 0, Omega >= 0 (template %lld)",
                            (long long)t);
            if (!(ap * om < 0.5)) return fail(c, FT_E_INVALID, "a_p * Omega must be < 1/2 (template %lld)", (long long)t);
            if (!(om * dt_abs + std::fabs(pb) < 1.5e6))
                return fail(c, FT_E_UNSUPPORTED, "orbital phase beyond 1.5e6 rad (template %lld)", (long long)t);
            aw_max = std::max(aw_max, ap * om);
        }
    }
    const double x_max = (f0_max + c_max) * (1.0 + c->vmax + aw_max) * c->t_sft;
    if (!(x_max < 2147483000.0)) return fail(c, FT_E_UNSUPPORTED, "track frequencies above 2^31/T_sft");
    bool bin_range_ok = false;
    if (binary) {
        bin_range_ok = true;
        for (int64_t t = 0; t < n0 && bin_range_ok; ++t)
            bin_range_ok = binary_range_ok(c, c->f0_h[t], c->f0_h[t], c->ap_h[t] * c->omega_h[t]);
    }

    // upload
    if ((e = ensure(&c->d_f0, &c->cap_f0, (size_t)n0)) != hipSuccess ||
        (e = ensure(&c->d_f1, &c->cap_f1, (size_t)n1)) != hipSuccess ||
        (e = ensure(&c->d_sky, &c->cap_sky, (size_t)ns * 3)) != hipSuccess ||
        (e = ensure(&c->d_stats, &c->cap_stats, (size_t)n_t)) != hipSuccess)
        return hip_fail(c, e, "alloc bank");
    if (grid) {
        const bool same_sky = c->sky_order_valid && c->sky_order_of.size() == c->sky_h.size() &&
                              std::memcmp(c->sky_order_of.data(), c->sky_h.data(), c->sky_h.size() * sizeof(double)) == 0;
        if (!same_sky) {
            c->sky_order_valid = false;
            sky_order(c->sky_h, ns, c->perm_h);
            c->sky_tile_h.resize((size_t)ns * 3);
            for (int64_t s = 0; s < ns; ++s)
                for (int d = 0; d < 3; ++d) c->sky_tile_h[3 * s + d] = c->sky_h[3 * (size_t)c->perm_h[s] + d];
            if ((e = ensure(&c->d_sky_tile, &c->cap_sky_tile, (size_t)ns * 3)) != hipSuccess ||
                (e = ensure(&c->d_perm, &c->cap_perm, (size_t)ns)) != hipSuccess)
                return hip_fail(c, e, "alloc sky order");
            e = hipMemcpyAsync(c->d_sky_tile, c->sky_tile_h.data(), ns * 3 * sizeof(double), hipMemcpyHostToDevice,
                               c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->d_perm, c->perm_h.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "upload sky order");
            c->sky_order_of = c->sky_h;
            c->sky_order_valid = true;
        }
    }
    e = hipMemcpyAsync(c->d_f0, c->f0_h.data(), n0 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_f1, c->f1_h.data(), n1 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_sky, c->sky_h.data(), ns * 3 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && binary) {
        if ((e = ensure(&c->d_bin, &c->cap_bin, (size_t)n0 * 3)) != hipSuccess) return hip_fail(c, e, "alloc binary bank");
        e = hipMemcpyAsync(c->d_bin, c->ap_h.data(), n0 * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->d_bin + n0, c->omega_h.data(), n0 * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->d_bin + 2 * n0, c->phib_h.data(), n0 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    }
    if (e == hipSuccess) e = launch_dt(c->d_tmid, t_ref, c->d_dt, c->n_sft, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "upload bank");

    run = EvalRun{};
    run.power = c->d_power;
    run.power_w = c->has_weight ? c->d_power_w : c->d_power;
    run.weight = c->has_weight ? c->d_weight : nullptr;
    run.dt = c->d_dt;
    run.v = c->d_v;
    run.f0 = c->d_f0;
    run.f1 = c->d_f1;
    run.sky = c->d_sky;
    run.v32 = c->d_v32;
    run.ap = binary ? c->d_bin : nullptr;
    run.omega = binary ? c->d_bin + n0 : nullptr;
    run.phib = binary ? c->d_bin + 2 * n0 : nullptr;
    run.sky_tile = grid ? c->d_sky_tile : nullptr;
    run.sky_perm = grid ? c->d_perm : nullptr;
    run.stats = c->d_stats;
    run.err = c->d_err;
    run.n_sft = c->n_sft;
    run.n_bins = c->n_bins;
    run.first_bin = (int32_t)c->first_bin;
    run.n_f0 = (int32_t)(grid ? n0 : 0);
    run.n_f1 = (int32_t)(grid ? n1 : 0);
    run.n_sky = (int32_t)(grid ? ns : 0);
    run.n_list = grid ? 0 : n0;
    run.t_sft = c->t_sft;
    run.vmax = c->vmax;
    if (binary) {
        ft_status stc = binary_cos_delta(c, run.cos_delta);
        if (stc != FT_OK) return stc;
        run.range_ok = bin_range_ok ? 1 : 0;
    }
    // bounds used by the grid kernel
    if (grid) guard_params(c->f0_h.data(), n0, f0_max, x_max, c->vmax, c->t_sft, run.dT, run.eta);
    (void)dt_min;
    return FT_OK;
}

static ft_status ensure_select(ft_ctx c, int n_seg, int k, int64_t n_seg_map, int64_t cap)
{
    hipError_t e;
    if ((e = ensure(&c->d_hist, &c->cap_hist, (size_t)n_seg * 256)) != hipSuccess ||
        (e = ensure(&c->d_state, &c->cap_state, (size_t)n_seg * 8)) != hipSuccess ||
        (e = ensure(&c->d_cnt, &c->cap_cnt, (size_t)n_seg)) != hipSuccess ||
        (e = ensure(&c->d_off, &c->cap_off, (size_t)n_seg + 1)) != hipSuccess ||
        (e = ensure(&c->d_fill, &c->cap_fill, (size_t)n_seg)) != hipSuccess ||
        (e = ensure(&c->d_cand, &c->cap_cand, (size_t)cap)) != hipSuccess ||
        (e = ensure(&c->d_cand_s64, &c->cap_cand_s64, (size_t)cap)) != hipSuccess ||
        (e = ensure(&c->d_cand_mom, &c->cap_cand_mom, (size_t)cap * 2)) != hipSuccess ||
        (e = ensure(&c->d_seg, &c->cap_seg, (size_t)n_seg_map)) != hipSuccess ||
        (e = ensure(&c->d_out, &c->cap_out, (size_t)n_seg * k)) != hipSuccess ||
        (e = ensure(&c->d_nout, &c->cap_nout, (size_t)n_seg)) != hipSuccess)
        return hip_fail(c, e, "alloc selection buffers");
    return FT_OK;
}

static SelectBufs select_bufs(ft_ctx c, int64_t cap, int stat)
{
    SelectBufs b;
    b.hist = c->d_hist;
    b.state = c->d_state;
    b.cnt = c->d_cnt;
    b.off = c->d_off;
    b.fill = c->d_fill;
    b.cand = c->d_cand;
    b.cand_s64 = c->d_cand_s64;
    b.cand_mom = c->d_cand_mom;
    b.seg_of_f0 = c->d_seg;
    b.out = c->d_out;
    b.n_out = c->d_nout;
    b.mu_sigma = stat == FT_STAT_NUMBER_COUNT ? c->d_mu_sigma_nc : c->d_mu_sigma;
    b.cap = cap;
    return b;
}

// Shape class of a GRID call for the tile cache.
static std::vector<int64_t> plain_tune_key(ft_ctx c, int64_t n0, int64_t n1, int64_t ns, bool uniform)
{
    const double dop = c->f0_h[(size_t)n0 - 1] * c->vmax * c->t_sft;
    return {0, n0, n1, (int64_t)c->n_sft, (int64_t)floor_log2(ns), (int64_t)dop, uniform ? 1 : 0};
}

static hipError_t launch_grid(const EvalRun &run, int tile, const WindowPlan *tail, hipStream_t s);

// Times the candidate tiles on a sample of the Doppler-ordered sky (blocks
// spread over the whole order, about 1e12 evaluations) and returns the
// fastest in best (0-based; -1 when no candidate's window fits in LDS).  Each
// candidate runs as a call would run it: with its f1-tail companion when its
// JT does not divide n_f1.
static ft_status tune_plain(ft_ctx c, const EvalRun &run, double dt_absmax, bool uniform, int &best)
{
    const auto t_start = std::chrono::steady_clock::now();
    best = -1;
    const int64_t n0 = run.n_f0, n1 = run.n_f1, ns = run.n_sky;
    const double per_sky = (double)n0 * (double)n1 * (double)c->n_sft;
    // the sample, about 1e12 evaluations in one launch: blocks of 64
    // consecutive points of the Doppler-ordered sky (a tile keeps its
    // neighbours) at evenly spaced positions over the whole order, since the
    // share of whole-wave steps, and with it the ranking of the tiles,
    // changes with the sky region.  Its size keeps the partly filled last
    // round of workgroups of each dispatch (a tile and its f1-tail companion
    // are two) below a few percent of the time.
    constexpr int64_t kBlock = 64;
    int64_t n_s = (int64_t)std::ceil(1e12 / per_sky);
    n_s = (n_s + kBlock - 1) / kBlock * kBlock;
    const double *smp_sky = run.sky_tile;
    const int32_t *smp_perm = run.sky_perm;
    std::vector<double> st_h;
    std::vector<int32_t> sp_h;
    if (n_s >= ns) {
        n_s = ns;
    } else {
        const int64_t n_blk = n_s / kBlock;
        st_h.resize((size_t)n_s * 3);
        sp_h.resize((size_t)n_s);
        for (int64_t b = 0; b < n_blk; ++b) {
            const int64_t start = n_blk > 1 ? (ns - kBlock) * b / (n_blk - 1) : 0;
            for (int64_t i = 0; i < kBlock; ++i) {
                for (int d = 0; d < 3; ++d) st_h[(size_t)(3 * (b * kBlock + i) + d)] = c->sky_tile_h[(size_t)(3 * (start + i) + d)];
                sp_h[(size_t)(b * kBlock + i)] = c->perm_h[(size_t)(start + i)];
            }
        }
        hipError_t e = ensure(&c->d_tune_sky, &c->cap_tune_sky, (size_t)n_s * 3);
        if (e == hipSuccess) e = ensure(&c->d_tune_perm, &c->cap_tune_perm, (size_t)n_s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->d_tune_sky, st_h.data(), st_h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->d_tune_perm, sp_h.data(), sp_h.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                               c->stream);
        // the host vectors are released on every return below: complete the copies
        hipError_t es = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) e = es;
        if (e != hipSuccess) return hip_fail(c, e, "tile tuning sample");
        smp_sky = c->d_tune_sky;
        smp_perm = c->d_tune_perm;
    }
    struct Trial {
        int tile;
        EvalRun r;
        WindowPlan tail;  // tile -1: no f1-tail dispatch
    };
    std::vector<Trial> trials;
    for (int id : tune_candidates((double)n0, (double)n1, uniform)) {
        const WindowPlan wp = plan_window(c->f0_h.data(), n0, c->f1_h.data(), n1, c->sky_tile_h.data(), ns, dt_absmax,
                                          c->vmax, c->t_sft, id);
        if (wp.tile < 0) continue;
        EvalRun r = run;
        r.wt = wp.wt;
        r.wtp = wp.wtp;
        r.tiles_f0 = wp.tiles_f0;
        r.tiles_f1 = wp.tiles_f1;
        r.sky_tile = smp_sky;
        r.sky_perm = smp_perm;
        r.n_sky = (int32_t)n_s;
        r.tiles_sky = (int32_t)((n_s + tile_cfg(id).NW - 1) / tile_cfg(id).NW);
        WindowPlan tail;
        const int jt = tile_cfg(id).JT;
        const int rem = (int)(n1 % jt);
        const int comp = rem && n1 > jt ? tile_companion(id, rem) : -1;
        if (comp >= 0 && (!run.sky_norm || tile_has_sky_weights(comp))) {
            tail = plan_window(c->f0_h.data(), n0, c->f1_h.data() + (n1 - rem), rem, c->sky_tile_h.data(), ns,
                               dt_absmax, c->vmax, c->t_sft, comp);
            if (tail.tile >= 0) tail.tiles_sky = (int32_t)((n_s + tile_cfg(comp).NW - 1) / tile_cfg(comp).NW);
        }
        trials.push_back({id, r, tail});
    }
    c->tune_log.clear();
    if (trials.empty()) return FT_OK;
    // the first launch also brings the clocks up; it is not timed
    auto tail_of = [](const Trial &t) { return t.tail.tile >= 0 ? &t.tail : nullptr; };
    auto launch_sample = [&](const Trial &t) { return launch_grid(t.r, t.tile, tail_of(t), c->stream); };
    hipError_t e = launch_sample(trials[0]);
    std::vector<float> ms(trials.size(), 0.f);
    for (size_t i = 0; i < trials.size() && e == hipSuccess; ++i) {
        e = hipEventRecord(c->ev[0], c->stream);
        if (e == hipSuccess) e = launch_sample(trials[i]);
        if (e == hipSuccess) e = hipEventRecord(c->ev[1], c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(c->ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms[i], c->ev[0], c->ev[1]);
    }
    if (e != hipSuccess) return hip_fail(c, e, "tile tuning");
    size_t bi = 0;
    for (size_t i = 1; i < trials.size(); ++i)
        if (ms[i] < ms[bi]) bi = i;
    best = trials[bi].tile;
    const double evals = per_sky * (double)n_s;
    for (size_t i = 0; i < trials.size(); ++i) {
        ft_tune_entry t{};
        t.klass = 0;
        t.tile = trials[i].tile + 1;
        t.chosen = i == bi;
        t.evals_per_s = ms[i] > 0.f ? evals / (ms[i] * 1e-3) : 0.0;
        t.sample_evals = evals;
        c->tune_log.push_back(t);
    }
    c->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return FT_OK;
}

// Evaluation options shared by every bank: validated, sub-band edges read.
// The statistic's options (precision, sums, statistic, weights).
static ft_status check_stat_opts(ft_ctx c, const ft_eval_opts *opts)
{
    if (!opts) return fail(c, FT_E_INVALID, "opts is null");
    if (opts->precision != FT_INDEX_FP64)
        return fail(c, FT_E_UNSUPPORTED,
                    "ft_eval_templates computes canonical FP64 bins; the FP32/df64/guarded index "
                    "forms are available through ft_count_index_mismatches and ft_bins");
    if (opts->sum_mode != FT_SUM_BLOCKED && opts->sum_mode != FT_SUM_PLAIN_FP32)
        return fail(c, FT_E_INVALID, "unknown sum_mode");
    if (opts->statistic != FT_STAT_POWER && opts->statistic != FT_STAT_NUMBER_COUNT)
        return fail(c, FT_E_INVALID, "unknown statistic %d", opts->statistic);
    if (opts->weights != FT_WEIGHTS_SFT && opts->weights != FT_WEIGHTS_SKY)
        return fail(c, FT_E_INVALID, "unknown weights %d", opts->weights);
    return FT_OK;
}

static ft_status check_eval_opts(ft_ctx c, const ft_eval_opts *opts, std::vector<double> &edges)
{
    ft_status st = check_stat_opts(c, opts);
    if (st != FT_OK) return st;
    if (opts->k < 1 || opts->k > 65536) return fail(c, FT_E_INVALID, "k must be in [1, 65536]");
    if (opts->n_sub < 1 || opts->n_sub > 4096) return fail(c, FT_E_INVALID, "n_sub must be in [1, 4096]");
    if (!opts->sub_edges) return fail(c, FT_E_INVALID, "sub_edges is null");
    if (opts->tile < FT_TILE_TUNE || opts->tile > tile_count()) return fail(c, FT_E_INVALID, "unknown tile %d", opts->tile);
    if (fetch(edges, opts->sub_edges, (size_t)opts->n_sub + 1) != hipSuccess)
        return fail(c, FT_E_INVALID, "cannot read sub_edges");
    for (size_t j = 0; j < edges.size(); ++j) {
        if (!is_finite(edges[j])) return fail(c, FT_E_INVALID, "sub_edges must be finite");
        if (j > 0 && !(edges[j] > edges[j - 1])) return fail(c, FT_E_INVALID, "sub_edges must be strictly increasing");
    }
    return FT_OK;
}

static ft_status launch_eval_select(ft_ctx c, EvalRun &run, bool grid, int tile, int64_t n_t, int64_t n_seg_map,
                                    const ft_eval_opts *opts, const std::vector<double> &edges, float *stats,
                                    const WindowPlan *tail = nullptr);

// The statistic's tables (number count: the indicator tables) and, for
// sky-dependent weights, the per-sky buffers the evaluation fills.
static ft_status apply_stat_weights(ft_ctx c, const ft_eval_opts *opts, bool grid, int64_t n_sky, EvalRun &run)
{
    run.stat = opts->statistic;
    if (opts->statistic == FT_STAT_NUMBER_COUNT) {
        ft_status st = ensure_nc(c);
        if (st != FT_OK) return st;
        run.power = c->d_ind;
        run.power_w = c->has_weight ? c->d_ind_w : c->d_ind;
    }
    if (opts->weights == FT_WEIGHTS_SKY) {
        if (!grid && !run.ap)
            return fail(c, FT_E_UNSUPPORTED, "sky-dependent weights are available for GRID and BINARY banks");
        if (!c->have_arms) return fail(c, FT_E_STATE, "sky-dependent weights need ft_set_arms");
        if (!grid) {  // binary banks: weights normalised per template in the kernels
            run.arms = c->d_arms;
            return FT_OK;
        }
        hipError_t e;
        if ((e = ensure(&c->d_sky_norm, &c->cap_sky_norm, (size_t)n_sky)) != hipSuccess ||
            (e = ensure(&c->d_sky_ms, &c->cap_sky_ms, (size_t)n_sky * 2)) != hipSuccess)
            return hip_fail(c, e, "alloc sky weights");
        run.arms = c->d_arms;
        run.sky_norm = c->d_sky_norm;
        run.sky_ms = c->d_sky_ms;
    }
    return FT_OK;
}

// Tiles with a sky-weighted form: the run tile for uniform f0 grids and the
// single-f0 tile otherwise.
constexpr int kSkyTileRun = 17;  // L5_J4_W4_K8_O4
constexpr int kSkyTileOne = 1;   // L1_J4_W4_K16

ft_status ft_eval_templates(ft_ctx c, const ft_bank *bank, double t_ref, const ft_eval_opts *opts,
                            float *stats)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    std::vector<double> edges;
    ft_status st0 = check_eval_opts(c, opts, edges);
    if (st0 != FT_OK) return st0;
    EvalRun run;
    bool grid;
    int64_t n_t;
    ft_status st = prepare_bank(c, bank, t_ref, run, grid, n_t);
    if (st != FT_OK) return st;
    st = apply_stat_weights(c, opts, grid, grid ? bank->n_sky : 0, run);
    if (st != FT_OK) return st;
    const bool sky = run.sky_norm != nullptr;
    run.sum_mode = opts->sum_mode;
    run.precision = opts->precision;

    // tile choice and LDS window for the grid kernel
    int tile = -1;
    WindowPlan tail;  // the tile of the last f1 values (tile -1: none)
    if (grid) {
        const int64_t n0 = bank->n_f0, n1 = bank->n_f1, ns = bank->n_sky;
        const bool uniform = run.eta < 1e-4;
        double dt_absmax = 0.0;
        for (double t : c->t_mid_h) dt_absmax = std::max(dt_absmax, std::fabs(t - t_ref));
        if (sky) {
            if (opts->tile > 0 && !tile_has_sky_weights(opts->tile - 1))
                return fail(c, FT_E_INVALID, "tile %d has no form with sky-dependent weights", opts->tile);
            tile = opts->tile > 0 ? opts->tile - 1 : uniform ? kSkyTileRun : kSkyTileOne;
        } else if (opts->tile > 0) {
            tile = opts->tile - 1;
        } else {
            const std::vector<int64_t> key = plain_tune_key(c, n0, n1, ns, uniform);
            const auto it = c->tune_cache.find(key);
            tile = -1;
            if (it != c->tune_cache.end()) {
                tile = it->second;
            } else if (opts->tile == FT_TILE_TUNE) {
                st = tune_plain(c, run, dt_absmax, uniform, tile);
                if (st != FT_OK) return st;
                if (tile >= 0) c->tune_cache[key] = tile;
            }
            if (tile < 0) tile = choose_tile(n0, n1, uniform);
        }
        if (tile_cfg(tile).L > 1 && !uniform) tile = kSkyTileOne;
        const WindowPlan wp = plan_window(c->f0_h.data(), n0, c->f1_h.data(), n1, c->sky_tile_h.data(), ns,
                                          dt_absmax, c->vmax, c->t_sft, tile);
        tile = wp.tile;  // -1: the window does not fit in LDS, use the direct kernel
        run.wt = wp.wt;
        run.wtp = wp.wtp;
        run.tiles_f0 = wp.tiles_f0;
        run.tiles_f1 = wp.tiles_f1;
        run.tiles_sky = wp.tiles_sky;
        if ((int64_t)run.tiles_f0 * run.tiles_f1 * run.tiles_sky >= 0x7fffffffLL)
            return fail(c, FT_E_UNSUPPORTED, "too many tiles");
        // When JT does not divide n_f1, the last rem f1 values go to the tile of
        // the same shape with JT = rem (no idle f1 slots); every tile shape gives
        // the same bits.
        if (tile >= 0) {
            const int jt = tile_cfg(tile).JT;
            const int rem = (int)(n1 % jt);
            const int comp = rem && n1 > jt ? tile_companion(tile, rem) : -1;
            if (comp >= 0 && (!run.sky_norm || tile_has_sky_weights(comp)))
                tail = plan_window(c->f0_h.data(), n0, c->f1_h.data() + (n1 - rem), rem, c->sky_tile_h.data(), ns,
                                   dt_absmax, c->vmax, c->t_sft, comp);
        }
    }

    return launch_eval_select(c, run, grid, tile, n_t, grid ? bank->n_f0 : n_t, opts, edges, stats,
                              tail.tile >= 0 ? &tail : nullptr);
}

// Launch sequence of an evaluation: clear flags, map sub-bands, evaluate,
// select, re-sum, rank (run fully prepared; n_seg_map = f0 values to map).
// Binary banks too small to fill the GPU with one lane per template (about
// 2^19 lanes are resident) split their SUM_BLOCK-SFT blocks over several
// workgroup rows; the per-block sums take n_list ceil(N / SUM_BLOCK) floats of
// context memory, at most 256 MB (else, or if that allocation fails, the bank
// is evaluated unsplit).  Either way the statistics are the same bits.
static hipError_t eval_binary(ft_ctx c, const EvalRun &run)
{
    constexpr int64_t kLanes = int64_t(1) << 19;
    constexpr size_t kMaxBytes = size_t(256) << 20;
    const int64_t n_blk = (run.n_sft + SUM_BLOCK - 1) / SUM_BLOCK;
    int n_seg = 1;
    if (!run.arms && run.sum_mode == FT_SUM_BLOCKED && run.n_list > 0 && run.n_list < kLanes && n_blk > 1 &&
        (size_t)n_blk * (size_t)run.n_list * sizeof(float) <= kMaxBytes) {
        n_seg = (int)std::min<int64_t>(n_blk, (kLanes + run.n_list - 1) / run.n_list);
        if (n_seg > 1 && ensure(&c->d_bsum, &c->cap_bsum, (size_t)(n_blk * run.n_list)) != hipSuccess) {
            (void)hipGetLastError();
            n_seg = 1;
        }
    }
    return launch_eval_binary(run, n_seg > 1 ? c->d_bsum : nullptr, n_seg, c->stream);
}

// Grid launch of `tile`; with `tail`, the f1 values past the last multiple of
// JT go to the tail's tile (a view of the same bank: f1 and stats shifted, the
// output rows keeping the whole bank's f1 count).
static hipError_t launch_grid(const EvalRun &run, int tile, const WindowPlan *tail, hipStream_t s)
{
    if (!tail) return launch_eval_grid(run, tile_cfg(tile), s);
    const TileCfg &cfg = tile_cfg(tile), &tcfg = tile_cfg(tail->tile);
    const int n_main = run.n_f1 - tcfg.JT;
    EvalRun a = run;
    a.n_f1 = n_main;
    a.n_f1_stride = run.n_f1;
    a.tiles_f1 = n_main / cfg.JT;
    EvalRun b = run;
    b.f1 = run.f1 + n_main;
    b.n_f1 = tcfg.JT;
    b.n_f1_stride = run.n_f1;
    b.stats = run.stats + (int64_t)n_main * run.n_f0;
    b.wt = tail->wt;
    b.wtp = tail->wtp;
    b.tiles_f0 = tail->tiles_f0;
    b.tiles_f1 = tail->tiles_f1;
    b.tiles_sky = tail->tiles_sky;
    hipError_t e = launch_eval_grid(a, cfg, s);
    if (e == hipSuccess) e = launch_eval_grid(b, tcfg, s);
    return e;
}

static ft_status launch_eval_select(ft_ctx c, EvalRun &run, bool grid, int tile, int64_t n_t, int64_t n_seg_map,
                                    const ft_eval_opts *opts, const std::vector<double> &edges, float *stats,
                                    const WindowPlan *tail)
{
    hipError_t e;
    ft_status st;
    const int n_seg = opts->n_sub;
    const int k = opts->k;
    // first guess of the candidate buffer: 64 per toplist slot, never more than
    // the templates themselves nor 2^26 entries (ft_sync regrows it to the
    // exact count when the threshold ties many templates)
    const int64_t cap = std::min<int64_t>({std::max<int64_t>(65536, (int64_t)64 * k * n_seg),
                                           std::max<int64_t>(n_t, 1), (int64_t)1 << 26});
    st = ensure_select(c, n_seg, k, n_seg_map, cap);
    if (st != FT_OK) return st;
    if ((e = ensure(&c->d_edges, &c->cap_edges, edges.size())) != hipSuccess) return hip_fail(c, e, "alloc edges");
    e = hipMemcpyAsync(c->d_edges, edges.data(), edges.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_fill_u32(c->d_err, 0u, 1, c->stream);
    if (e == hipSuccess) e = launch_subband_map(c->d_f0, n_seg_map, c->d_edges, n_seg, c->d_seg, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev[0], c->stream);
    if (e == hipSuccess && run.sky_norm)
        e = launch_sky_moments(run.arms, run.weight, run.n_sft, run.sky, run.n_sky, opts->statistic, c->d_sky_norm,
                               c->d_sky_ms, c->d_err, c->stream);
    if (e == hipSuccess)
        e = run.ap ? eval_binary(c, run)
            : !grid ? launch_eval_list(run, c->stream)
            : tile < 0 ? launch_eval_grid_direct(run, c->stream) : launch_grid(run, tile, tail, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev[1], c->stream);
    const double N = (double)c->n_sft;
    // sky-dependent weights: one more rounding per term (the factor)
    const double rel_err = (opts->sum_mode == FT_SUM_BLOCKED ? 40.0 * std::ldexp(1.0, -24) + 4.0 * N * std::ldexp(1.0, -53)
                                                             : (N + 8.0) * std::ldexp(1.0, -24) + 4.0 * N * std::ldexp(1.0, -53)) +
                           (run.arms ? 4.0 * std::ldexp(1.0, -24) : 0.0);
    SelectBufs sb = select_bufs(c, cap, opts->statistic);
    if (e == hipSuccess) e = launch_select(run, grid, n_seg, k, rel_err, sb, c->stream);
    if (e == hipSuccess) e = launch_rescore_rank(run, grid, n_seg, k, sb, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev[2], c->stream);
    if (e == hipSuccess && stats)
        e = hipMemcpyAsync(stats, c->d_stats, (size_t)n_t * sizeof(float), hipMemcpyDefault, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "launch evaluation");
    c->have_eval = true;
    c->last_run = run;
    c->last_grid = grid;
    c->last_k = k;
    c->last_nsub = n_seg;
    c->last_cap = cap;
    c->last_rel_err = rel_err;
    c->last_tile = tile;
    c->last_stat = opts->statistic;
    return FT_OK;
}

static ft_status check_region(ft_ctx c, const ft_binary_region *reg)
{
    if (!reg) return fail(c, FT_E_INVALID, "region is null");
    const double v[12] = {reg->f0_lo,    reg->f0_hi,    reg->ap_lo,   reg->ap_hi,   reg->omega_lo, reg->omega_hi,
                          reg->alpha_lo, reg->alpha_hi, reg->sdec_lo, reg->sdec_hi, reg->phib_lo,  reg->phib_hi};
    for (double x : v)
        if (!is_finite(x)) return fail(c, FT_E_INVALID, "region bounds must be finite");
    if (!(reg->alpha_lo <= reg->alpha_hi) || !(reg->sdec_lo <= reg->sdec_hi) || !(reg->phib_lo <= reg->phib_hi) ||
        reg->sdec_lo < -1.0 || reg->sdec_hi > 1.0)
        return fail(c, FT_E_INVALID, "region needs lo <= hi and sin(declination) in [-1, 1]");
    if (!(std::fabs(reg->alpha_lo) < 1e6 && std::fabs(reg->alpha_hi) < 1e6 && std::fabs(reg->phib_lo) < 1e6 &&
          std::fabs(reg->phib_hi) < 1e6))
        return fail(c, FT_E_INVALID, "region angles must lie within 1e6 rad");
    if (!(reg->f0_lo > 0.0 && reg->f0_lo <= reg->f0_hi) || !(reg->ap_lo > 0.0 && reg->ap_lo <= reg->ap_hi) ||
        !(reg->omega_lo > 0.0 && reg->omega_lo <= reg->omega_hi))
        return fail(c, FT_E_INVALID, "region needs 0 < lo <= hi for f0, a_p and Omega");
    if (!(reg->ap_hi * reg->omega_hi < 0.5)) return fail(c, FT_E_INVALID, "region needs a_p * Omega < 1/2");
    return FT_OK;
}

ft_status ft_gen_binary_bank(ft_ctx c, const ft_binary_region *reg, uint64_t seed, int64_t first, int64_t n,
                             double *f0, double *sky_xyz, double *ap, double *omega, double *phib)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    ft_status st = check_region(c, reg);
    if (st != FT_OK) return st;
    if (n < 0 || first < 0 || first > INT64_MAX - n) return fail(c, FT_E_INVALID, "bad template range");
    if (n == 0) return FT_OK;
    if (!f0 || !sky_xyz || !ap || !omega || !phib) return fail(c, FT_E_INVALID, "output arrays must be non-null");
    if (n > (1LL << 31)) return fail(c, FT_E_UNSUPPORTED, "at most 2^31 templates per call");
    hipError_t e;
    if ((e = ensure(&c->d_genbank, &c->cap_genbank, (size_t)n * 7)) != hipSuccess) return hip_fail(c, e, "alloc bank");
    double *d = c->d_genbank;
    e = launch_gen_binary_bank(*reg, seed, first, n, d, d + n, d + 4 * n, d + 5 * n, d + 6 * n, c->stream);
    const std::pair<double *, int64_t> outs[5] = {{f0, 0}, {sky_xyz, n}, {ap, 4 * n}, {omega, 5 * n}, {phib, 6 * n}};
    for (int q = 0; q < 5 && e == hipSuccess; ++q)
        e = hipMemcpyAsync(outs[q].first, d + outs[q].second, (q == 1 ? 3 : 1) * n * sizeof(double), hipMemcpyDefault,
                           c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "generate bank");
    return FT_OK;
}

// Random binary bank generated on the device (with each template's hyperbox
// when div is given) and the evaluation run over it.
static ft_status binary_random_run(ft_ctx c, const ft_binary_region *reg, uint64_t seed, int64_t n, double t_ref,
                                   const ft_eval_opts *opts, EvalRun &run, const BoxDiv *div, int32_t *box)
{
    ft_status st = check_region(c, reg);
    if (st != FT_OK) return st;
    if (!c->have_sfts || !c->have_vel) return fail(c, FT_E_STATE, "ft_set_sfts and ft_set_velocities must come first");
    if (!is_finite(t_ref)) return fail(c, FT_E_INVALID, "t_ref must be finite");
    if (n < 1 || n >= (1LL << 31)) return fail(c, FT_E_UNSUPPORTED, "n must be in [1, 2^31)");
    if (c->n_bins >= (1 << 28)) return fail(c, FT_E_UNSUPPORTED, "binary banks need tables of fewer than 2^28 columns");
    double dt_abs = 0.0;
    for (double t : c->t_mid_h) dt_abs = std::max(dt_abs, std::fabs(t - t_ref));
    if (!(reg->omega_hi * dt_abs + std::max(std::fabs(reg->phib_lo), std::fabs(reg->phib_hi)) < 1.5e6))
        return fail(c, FT_E_UNSUPPORTED, "orbital phase beyond 1.5e6 rad");
    const double x_max = reg->f0_hi * (1.0 + c->vmax + reg->ap_hi * reg->omega_hi) * c->t_sft;
    if (!(x_max < 2147483000.0)) return fail(c, FT_E_UNSUPPORTED, "track frequencies above 2^31/T_sft");
    hipError_t e;
    if ((e = ensure(&c->d_f0, &c->cap_f0, (size_t)n)) != hipSuccess || (e = ensure(&c->d_sky, &c->cap_sky, (size_t)n * 3)) != hipSuccess ||
        (e = ensure(&c->d_bin, &c->cap_bin, (size_t)n * 3)) != hipSuccess ||
        (e = ensure(&c->d_stats, &c->cap_stats, (size_t)n)) != hipSuccess)
        return hip_fail(c, e, "alloc bank");
    e = launch_gen_binary_bank(*reg, seed, 0, n, c->d_f0, c->d_sky, c->d_bin, c->d_bin + n, c->d_bin + 2 * n, c->stream,
                               div, box);
    if (e == hipSuccess) e = launch_dt(c->d_tmid, t_ref, c->d_dt, c->n_sft, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "generate bank");
    run = EvalRun{};
    run.power = c->d_power;
    run.power_w = c->has_weight ? c->d_power_w : c->d_power;
    run.weight = c->has_weight ? c->d_weight : nullptr;
    run.dt = c->d_dt;
    run.v = c->d_v;
    run.v32 = c->d_v32;
    run.f0 = c->d_f0;
    run.f1 = nullptr;
    run.sky = c->d_sky;
    run.ap = c->d_bin;
    run.omega = c->d_bin + n;
    run.phib = c->d_bin + 2 * n;
    run.stats = c->d_stats;
    run.err = c->d_err;
    run.n_sft = c->n_sft;
    run.n_bins = c->n_bins;
    run.first_bin = (int32_t)c->first_bin;
    run.n_list = n;
    run.t_sft = c->t_sft;
    run.vmax = c->vmax;
    run.sum_mode = opts->sum_mode;
    run.precision = opts->precision;
    st = binary_cos_delta(c, run.cos_delta);
    if (st != FT_OK) return st;
    run.range_ok = binary_range_ok(c, reg->f0_lo, reg->f0_hi, reg->ap_hi * reg->omega_hi) ? 1 : 0;
    return apply_stat_weights(c, opts, false, 0, run);
}

ft_status ft_eval_binary_random(ft_ctx c, const ft_binary_region *reg, uint64_t seed, int64_t n, double t_ref,
                                const ft_eval_opts *opts, float *stats)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    std::vector<double> edges;
    ft_status st = check_eval_opts(c, opts, edges);
    if (st != FT_OK) return st;
    EvalRun run;
    st = binary_random_run(c, reg, seed, n, t_ref, opts, run, nullptr, nullptr);
    if (st != FT_OK) return st;
    return launch_eval_select(c, run, false, -1, n, n, opts, edges, stats);
}

ft_status ft_eval_binary_boxes(ft_ctx c, const ft_binary_region *reg, uint64_t seed, int64_t n, double t_ref,
                               const ft_box_partition *part, const ft_eval_opts *opts, ft_box_result *out,
                               float *stats)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    ft_status st = check_stat_opts(c, opts);
    if (st != FT_OK) return st;
    if (!part || !out) return fail(c, FT_E_INVALID, "part and out must be non-null");
    if (opts->weights != FT_WEIGHTS_SFT)
        return fail(c, FT_E_UNSUPPORTED, "the box search uses per-SFT weights (one noise mean and spread for all boxes)");
    BoxDiv div;
    int64_t n_boxes = 1;
    for (int d = 0; d < 6; ++d) {
        div.n[d] = part->n_div[d];
        if (div.n[d] < 1 || div.n[d] > (1 << 20)) return fail(c, FT_E_INVALID, "n_div[%d] must be in [1, 2^20]", d);
        n_boxes *= div.n[d];
        if (n_boxes > (1 << 26)) return fail(c, FT_E_INVALID, "more than 2^26 boxes");
    }
    if (n >= 1 && n < (1LL << 31)) {
        hipError_t e;
        if ((e = ensure(&c->d_box, &c->cap_box, (size_t)n)) != hipSuccess ||
            (e = ensure(&c->d_bcount, &c->cap_bcount, (size_t)n_boxes)) != hipSuccess ||
            (e = ensure(&c->d_bmax32, &c->cap_bmax32, (size_t)n_boxes)) != hipSuccess ||
            (e = ensure(&c->d_bmax64, &c->cap_bmax64, (size_t)n_boxes)) != hipSuccess ||
            (e = ensure(&c->d_bidx, &c->cap_bidx, (size_t)n_boxes)) != hipSuccess ||
            (e = ensure(&c->d_bout, &c->cap_bout, (size_t)n_boxes)) != hipSuccess ||
            (e = ensure(&c->d_bncand, &c->cap_bncand, 2)) != hipSuccess)
            return hip_fail(c, e, "alloc box buffers");
    }
    EvalRun run;
    st = binary_random_run(c, reg, seed, n, t_ref, opts, run, &div, c->d_box);
    if (st != FT_OK) return st;
    c->have_eval = false;  // the bank and statistics are replaced
    const double N = (double)c->n_sft;
    const double rel_err = opts->sum_mode == FT_SUM_BLOCKED ? 40.0 * std::ldexp(1.0, -24) + 4.0 * N * std::ldexp(1.0, -53)
                                                            : (N + 8.0) * std::ldexp(1.0, -24) + 4.0 * N * std::ldexp(1.0, -53);
    int64_t cap = std::max<int64_t>(65536, 4 * n_boxes);
    for (int attempt = 0; attempt < 2; ++attempt) {
        hipError_t e;
        if ((e = ensure(&c->d_bcand, &c->cap_bcand, (size_t)cap)) != hipSuccess ||
            (e = ensure(&c->d_bcand_s64, &c->cap_bcand_s64, (size_t)cap)) != hipSuccess)
            return hip_fail(c, e, "alloc box candidates");
        BoxBufs bb{c->d_box, c->d_bmax32, c->d_bcount, c->d_bmax64, c->d_bidx, c->d_bcand, c->d_bcand_s64, c->d_bncand, cap};
        e = launch_fill_u32(c->d_err, 0u, 1, c->stream);
        if (e == hipSuccess && attempt == 0) e = eval_binary(c, run);
        if (e == hipSuccess) e = launch_box_max(run, n, n_boxes, bb, rel_err, c->stream);
        uint32_t n_cand[2] = {0, 0};
        if (e == hipSuccess) e = hipMemcpyAsync(n_cand, c->d_bncand, sizeof n_cand, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "box maxima");
        if ((int64_t)n_cand[1] > cap) {  // grow and redo the candidate pass
            cap = (int64_t)n_cand[1] + 1024;
            continue;
        }
        const double *ms = opts->statistic == FT_STAT_NUMBER_COUNT ? c->d_mu_sigma_nc : c->d_mu_sigma;
        e = launch_box_pick(run, n_boxes, bb, ms, c->d_bout, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(out, c->d_bout, (size_t)n_boxes * sizeof(ft_box_result), hipMemcpyDefault, c->stream);
        if (e == hipSuccess && stats)
            e = hipMemcpyAsync(stats, c->d_stats, (size_t)n * sizeof(float), hipMemcpyDefault, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "box selection");
        return sync_and_check(c);
    }
    return fail(c, FT_E_INTERNAL, "box candidate buffer overflow after growth");
}

ft_status ft_sync(ft_ctx c)
{
    if (!c) return FT_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    ft_status st = sync_and_check(c);
    if (st != FT_OK || !c->have_eval) return st;
    // Grow the candidate buffer and redo the compaction if it overflowed.
    uint32_t flags = 0;
    hipMemcpy(&flags, c->d_err, sizeof flags, hipMemcpyDeviceToHost);
    if (flags & ERR_CAND_OVERFLOW) {
        uint32_t total = 0;
        hipMemcpy(&total, c->d_off + c->last_nsub, sizeof total, hipMemcpyDeviceToHost);
        // the per-sub-band offsets are 32-bit and saturate at 2^32 - 1
        if (total == 0xffffffffu)
            return fail(c, FT_E_UNSUPPORTED, "2^32 - 1 or more toplist candidates (the K-th largest statistic ties too many templates)");
        const EvalRun &lr = c->last_run;
        const int64_t n_last = c->last_grid ? (int64_t)lr.n_f0 * lr.n_f1 * lr.n_sky : lr.n_list;
        const int64_t cap = std::min<int64_t>((int64_t)total + 1024, std::max<int64_t>(n_last, 1));
        st = ensure_select(c, c->last_nsub, c->last_k, c->last_grid ? c->last_run.n_f0 : c->last_run.n_list, cap);
        if (st != FT_OK) return st;
        c->last_run.err = c->d_err;
        c->last_cap = cap;
        SelectBufs sb = select_bufs(c, cap, c->last_stat);
        hipError_t e = launch_fill_u32(c->d_err, 0u, 1, c->stream);
        if (e == hipSuccess) e = launch_select(c->last_run, c->last_grid, c->last_nsub, c->last_k, c->last_rel_err, sb, c->stream);
        if (e == hipSuccess) e = launch_rescore_rank(c->last_run, c->last_grid, c->last_nsub, c->last_k, sb, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "relaunch selection");
        st = sync_and_check(c);
        if (st != FT_OK) return st;
        hipMemcpy(&flags, c->d_err, sizeof flags, hipMemcpyDeviceToHost);
        if (flags & ERR_CAND_OVERFLOW) return fail(c, FT_E_INTERNAL, "candidate buffer overflow after growth");
    }
    return FT_OK;
}

ft_status ft_toplist(ft_ctx c, int32_t sub, ft_candidate *out, int32_t *n_out)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (!c->have_eval) return fail(c, FT_E_STATE, "no evaluation to read a toplist from");
    if (sub < 0 || sub >= c->last_nsub) return fail(c, FT_E_INVALID, "sub-band %d out of range", sub);
    if (!out || !n_out) return fail(c, FT_E_INVALID, "out and n_out must be non-null");
    ft_status st = ft_sync(c);
    if (st != FT_OK) return st;
    int32_t n = 0;
    hipError_t e = hipMemcpy(&n, c->d_nout + sub, sizeof n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && n > 0)
        e = hipMemcpy(out, c->d_out + (size_t)sub * c->last_k, (size_t)n * sizeof(ft_candidate), hipMemcpyDefault);
    if (e != hipSuccess) return hip_fail(c, e, "copy toplist");
    *n_out = n;
    return FT_OK;
}

ft_status ft_binary_cos_mode(ft_ctx c, int32_t mode, double *hw_err)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (mode != 0 && mode != 1) return fail(c, FT_E_INVALID, "mode must be 0 (auto) or 1 (library polynomial)");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    c->cos_mode = 0;
    double delta;
    ft_status st = binary_cos_delta(c, delta);  // measures once
    c->cos_mode = mode;
    if (st != FT_OK) return st;
    if (hw_err) *hw_err = c->hw_cos_err;
    return FT_OK;
}

ft_status ft_toplist_number_count(ft_ctx c, int32_t sub, double *nc_out, double *z_out, int32_t *n_out)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (!c->have_eval) return fail(c, FT_E_STATE, "no evaluation to read a toplist from");
    if (sub < 0 || sub >= c->last_nsub) return fail(c, FT_E_INVALID, "sub-band %d out of range", sub);
    if (!nc_out || !n_out) return fail(c, FT_E_INVALID, "nc_out and n_out must be non-null");
    ft_status st = ft_sync(c);
    if (st == FT_OK) st = ensure_nc(c);
    if (st != FT_OK) return st;
    hipError_t e = ensure(&c->d_top_nc, &c->cap_top_nc, (size_t)c->last_k * 3);
    if (e != hipSuccess) return hip_fail(c, e, "alloc number counts");
    EvalRun r = c->last_run;
    r.power = c->d_ind;  // the weights (per SFT or per sky point) stay those of the evaluation
    int32_t n = 0;
    e = launch_rescore_entries(r, c->last_grid, c->d_out + (size_t)sub * c->last_k, c->d_nout + sub, c->d_top_nc,
                               c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&n, c->d_nout + sub, sizeof n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    std::vector<double> h((size_t)std::max(n, 0) * 3);
    if (e == hipSuccess && n > 0)
        e = hipMemcpyAsync(h.data(), c->d_top_nc, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "number counts of the toplist");
    st = sync_and_check(c);
    if (st != FT_OK) return st;
    // the critical ratio of the number count, moments from the entry's own weights
    const double p = std::exp(-1.6);
    std::vector<double> nc((size_t)std::max(n, 0)), z(nc.size());
    for (int32_t i = 0; i < n; ++i) {
        nc[(size_t)i] = h[3 * (size_t)i];
        z[(size_t)i] = (h[3 * (size_t)i] - p * h[3 * (size_t)i + 1]) / std::sqrt(p * (1.0 - p) * h[3 * (size_t)i + 2]);
    }
    if (n > 0) {
        e = hipMemcpy(nc_out, nc.data(), nc.size() * sizeof(double), hipMemcpyDefault);
        if (e == hipSuccess && z_out) e = hipMemcpy(z_out, z.data(), z.size() * sizeof(double), hipMemcpyDefault);
        if (e != hipSuccess) return hip_fail(c, e, "copy number counts");
    }
    *n_out = n;
    return FT_OK;
}

ft_status ft_last_eval_info(ft_ctx c, ft_eval_info *info)
{
    if (!c || !info) return FT_E_INVALID;
    if (!c->have_eval) return fail(c, FT_E_STATE, "no evaluation yet");
    ft_status st = ft_sync(c);
    if (st != FT_OK) return st;
    memset(info, 0, sizeof *info);
    float ms = 0.f;
    hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
    info->eval_ms = ms;
    hipEventElapsedTime(&ms, c->ev[1], c->ev[2]);
    info->select_ms = ms;
    const EvalRun &r = c->last_run;
    info->n_templates = c->last_grid ? (int64_t)r.n_f0 * r.n_f1 * r.n_sky : r.n_list;
    info->n_evals = info->n_templates * (int64_t)r.n_sft;
    uint32_t total = 0;
    hipMemcpy(&total, c->d_off + c->last_nsub, sizeof total, hipMemcpyDeviceToHost);
    info->n_candidates = total;
    info->tile = c->last_tile + 1;
    info->window = c->last_grid ? r.wt : 0;
    return FT_OK;
}

ft_status ft_q_sample(ft_ctx c, const double *arms, int64_t n, const double *sky, const double *cos_iota,
                      const double *psi, double *q_out)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    if (!c->have_sfts) return fail(c, FT_E_STATE, "ft_set_sfts must come first");
    if (n < 0 || (n > 0 && (!arms || !sky || !cos_iota || !psi || !q_out))) return fail(c, FT_E_INVALID, "bad arguments");
    if (n == 0) return FT_OK;
    if (n >= (1LL << 31)) return fail(c, FT_E_UNSUPPORTED, "at most 2^31 - 1 samples per call");
    const int64_t N = c->n_sft;
    std::vector<double> ah, sh, ch, ph;
    if (fetch(ah, arms, (size_t)N * 6) != hipSuccess || fetch(sh, sky, (size_t)n * 3) != hipSuccess ||
        fetch(ch, cos_iota, (size_t)n) != hipSuccess || fetch(ph, psi, (size_t)n) != hipSuccess)
        return fail(c, FT_E_INVALID, "cannot read the inputs");
    for (double a : ah)
        if (!is_finite(a)) return fail(c, FT_E_INVALID, "arms hold a non-finite value");
    for (int64_t i = 0; i < n; ++i) {
        const double x = sh[3 * i], y = sh[3 * i + 1], z = sh[3 * i + 2];
        if (!is_finite(x) || !is_finite(y) || !is_finite(z) || std::fabs(std::sqrt(x * x + y * y + z * z) - 1.0) > 1e-12)
            return fail(c, FT_E_INVALID, "sky vectors must be finite unit vectors (sample %lld)", (long long)i);
        if (!is_finite(ch[i]) || ch[i] < -1.0 || ch[i] > 1.0 || !is_finite(ph[i]))
            return fail(c, FT_E_INVALID, "cos_iota must lie in [-1, 1] and psi be finite (sample %lld)", (long long)i);
    }
    // staging: arms | sky | cos_iota | psi | q
    const size_t need = (size_t)N * 6 + (size_t)n * 9;
    hipError_t e;
    if ((e = ensure(&c->d_qsample, &c->cap_qsample, need)) != hipSuccess) return hip_fail(c, e, "alloc q samples");
    double *d = c->d_qsample;
    double *d_arms = d, *d_sky = d + N * 6, *d_ci = d_sky + n * 3, *d_psi = d_ci + n, *d_q = d_psi + n;
    e = hipMemcpyAsync(d_arms, ah.data(), N * 6 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_sky, sh.data(), n * 3 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_ci, ch.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_psi, ph.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = launch_q_sample(d_arms, c->has_weight ? c->d_weight : nullptr, (int)N, c->t_sft, d_sky, d_ci, d_psi, n, d_q,
                            c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(q_out, d_q, n * 4 * sizeof(double), hipMemcpyDefault, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "q samples");
    return FT_OK;
}

ft_status ft_lib_sincos(ft_ctx c, const double *x, int64_t n, double *cos_out, double *sin_out)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    if (n < 0 || (n > 0 && (!x || (!cos_out && !sin_out)))) return fail(c, FT_E_INVALID, "bad arguments");
    if (n == 0) return FT_OK;
    std::vector<double> xh;
    if (fetch(xh, x, (size_t)n) != hipSuccess) return fail(c, FT_E_INVALID, "cannot read x");
    for (double v : xh)
        if (!is_finite(v) || !(std::fabs(v) < 1.5e6)) return fail(c, FT_E_INVALID, "x must be finite with |x| < 1.5e6");
    hipError_t e;
    if ((e = ensure(&c->d_sincos, &c->cap_sincos, (size_t)n * 3)) != hipSuccess) return hip_fail(c, e, "alloc sincos");
    e = hipMemcpyAsync(c->d_sincos, xh.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_lib_sincos(c->d_sincos, n, c->d_sincos + n, c->d_sincos + 2 * n, c->stream);
    if (e == hipSuccess && cos_out)
        e = hipMemcpyAsync(cos_out, c->d_sincos + n, n * sizeof(double), hipMemcpyDefault, c->stream);
    if (e == hipSuccess && sin_out)
        e = hipMemcpyAsync(sin_out, c->d_sincos + 2 * n, n * sizeof(double), hipMemcpyDefault, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "lib sincos");
    return FT_OK;
}

ft_status ft_bins(ft_ctx c, const ft_bank *bank, double t_ref, int32_t precision, int32_t *bins)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    if (!bins) return fail(c, FT_E_INVALID, "bins is null");
    if (precision < FT_INDEX_FP64 || precision > FT_INDEX_GUARDED_FP32) return fail(c, FT_E_INVALID, "unknown precision");
    if (bank && bank->kind != FT_BANK_LIST && bank->kind != FT_BANK_BINARY)
        return fail(c, FT_E_UNSUPPORTED, "ft_bins takes a LIST or BINARY bank");
    if (bank && bank->kind == FT_BANK_BINARY && precision != FT_INDEX_FP64)
        return fail(c, FT_E_UNSUPPORTED, "binary banks have canonical FP64 bins only");
    EvalRun run;
    bool grid;
    int64_t n_t;
    ft_status st = prepare_bank(c, bank, t_ref, run, grid, n_t);
    if (st != FT_OK) return st;
    const size_t n = (size_t)n_t * (size_t)c->n_sft;
    hipError_t e = ensure(&c->d_bins, &c->cap_bins, n);
    if (e == hipSuccess) e = launch_bins_list(run, precision, c->d_bins, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(bins, c->d_bins, n * sizeof(int32_t), hipMemcpyDefault, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "bins");
    c->have_eval = false;
    return FT_OK;
}

ft_status ft_count_index_mismatches(ft_ctx c, const ft_bank *bank, double t_ref, int32_t precision,
                                    int64_t *n_mismatch, int64_t *n_fallback)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    if (!n_mismatch) return fail(c, FT_E_INVALID, "n_mismatch is null");
    if (bank && bank->kind == FT_BANK_BINARY) return fail(c, FT_E_UNSUPPORTED, "the index study covers GRID and LIST banks");
    if (precision < FT_INDEX_FP64 || precision > FT_INDEX_GUARDED_FP32) return fail(c, FT_E_INVALID, "unknown precision");
    EvalRun run;
    bool grid;
    int64_t n_t;
    ft_status st = prepare_bank(c, bank, t_ref, run, grid, n_t);
    if (st != FT_OK) return st;
    unsigned long long cnt[2] = {0, 0};
    hipError_t e = hipMemsetAsync(c->d_count, 0, sizeof cnt, c->stream);
    if (e == hipSuccess) e = launch_count_mismatch(run, grid, precision, c->d_count, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(cnt, c->d_count, sizeof cnt, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "count mismatches");
    *n_mismatch = (int64_t)cnt[0];
    if (n_fallback) *n_fallback = (int64_t)cnt[1];
    c->have_eval = false;
    return FT_OK;
}

// True when p is device memory of `device` (memory the kernels may read).
static bool is_device_memory(const void *p, int device)
{
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice && attr.device == device;
}

ft_status ft_count_index_mismatches_noalloc(ft_ctx c, const ft_bank *bank, double t_ref, int32_t precision,
                                            int64_t *n_mismatch, int64_t *n_fallback)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    if (!n_mismatch) return fail(c, FT_E_INVALID, "n_mismatch is null");
    if (!bank) return fail(c, FT_E_INVALID, "bank is null");
    if (bank->kind != FT_BANK_GRID && bank->kind != FT_BANK_LIST)
        return fail(c, FT_E_UNSUPPORTED, "the index study covers GRID and LIST banks");
    if (precision < FT_INDEX_FP64 || precision > FT_INDEX_GUARDED_FP32) return fail(c, FT_E_INVALID, "unknown precision");
    if (!c->have_sfts || !c->have_vel) return fail(c, FT_E_STATE, "ft_set_sfts and ft_set_velocities must come first");
    if (c->n_sft > NOALLOC_MAX_SFT)
        return fail(c, FT_E_UNSUPPORTED, "%d SFTs: the no-allocation scratch holds at most %d", c->n_sft,
                    NOALLOC_MAX_SFT);
    if (!is_finite(t_ref)) return fail(c, FT_E_INVALID, "t_ref must be finite");
    const bool grid = bank->kind == FT_BANK_GRID;
    int64_t n0, n1, ns;
    if (grid) {
        n0 = bank->n_f0;
        n1 = bank->n_f1;
        ns = bank->n_sky;
        if (n0 < 1 || n1 < 1 || ns < 1) return fail(c, FT_E_INVALID, "grid sizes must be >= 1");
        if (n0 > 0x7fffffff || n1 > 0x7fffffff || ns > 0x7fffffff)
            return fail(c, FT_E_UNSUPPORTED, "grid dimension above 2^31-1");
        if (n0 * n1 > (1LL << 40) / ns) return fail(c, FT_E_UNSUPPORTED, "more than 2^40 templates in one call");
    } else {
        n0 = n1 = ns = bank->n_list;
        if (n0 < 1) return fail(c, FT_E_INVALID, "n_list must be >= 1");
    }
    if (!bank->f0 || !bank->f1 || !bank->sky_xyz) return fail(c, FT_E_INVALID, "bank arrays must be non-null");
    if (!is_device_memory(bank->f0, c->device) || !is_device_memory(bank->f1, c->device) ||
        !is_device_memory(bank->sky_xyz, c->device))
        return fail(c, FT_E_INVALID, "the no-allocation call reads the bank in place: f0, f1 and sky_xyz must be "
                                     "device memory of the context's GPU");
    void *scratch_ptr = noalloc_scratch_ptr(c->device);
    if (!scratch_ptr) return fail(c, FT_E_DEVICE, "no scratch address on device %d", c->device);
    EvalRun run{};
    run.v = c->d_v;
    run.f0 = bank->f0;
    run.f1 = bank->f1;
    run.sky = bank->sky_xyz;
    run.n_sft = c->n_sft;
    run.t_sft = c->t_sft;
    run.n_f0 = (int32_t)n0;
    run.n_f1 = (int32_t)n1;
    run.n_sky = (int32_t)ns;
    run.n_list = grid ? 0 : n0;
    unsigned long long cnt[2] = {0, 0};
    hipError_t e = launch_count_mismatch_noalloc(run, grid, precision, c->d_tmid, t_ref, scratch_ptr, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(cnt, scratch_ptr, sizeof cnt, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "count mismatches (no allocation)");
    *n_mismatch = (int64_t)cnt[0];
    if (n_fallback) *n_fallback = (int64_t)cnt[1];
    return FT_OK;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
namespace {

// Tile of one batch run: fewest wasted lanes over the tiles whose f1 tile
// suits small f1 sets.
int choose_batch_tile(int64_t n_f0, int64_t n_f1, bool uniform)
{
    const int with_runs[] = {15, 16, 2, 8};  // L3_J3, L5_J3, L3_J4, L5_J4
    const int plain[] = {14, 1};             // L1_J3, L1_J4
    double best = 1e30;
    int best_id = 14;
    auto consider = [&](int id) {
        const TileCfg &t = tile_cfg(id);
        const double f0w = std::ceil((double)n_f0 / (64.0 * t.L)) * 64.0 * t.L / (double)n_f0;
        const double f1w = std::ceil((double)n_f1 / t.JT) * t.JT / (double)n_f1;
        const double ops = t.L > 1 ? (7.0 + t.L) / t.L : 7.0;
        const double cost = f0w * f1w * ops;
        if (cost < best - 1e-9) {
            best = cost;
            best_id = id;
        }
    };
    if (uniform && n_f0 >= 32)
        for (int id : with_runs) consider(id);
    for (int id : plain) consider(id);
    return best_id;
}

struct BatchPlan {
    std::vector<EvalRun> runs;
    std::vector<GenRun> gen;
    std::vector<int> tile;                 // per run
    std::vector<int64_t> dt_prefix, stats_prefix, gen_prefix_sft, gen_prefix_elem, sky_prefix;
    std::vector<int32_t> sft_begin, perm;
    std::vector<double> tref, sky_tile;
    std::vector<std::vector<int2>> items;  // per tile id; index tile_count(): direct items
    std::vector<char> uniform;             // per run: the run-length guard applies
    std::vector<double> dt_absmax, vmax;   // per run: window inputs
    std::vector<int> group_wtp;            // per tile id: widest LDS row of its runs
    int small_chunk = 8;                   // f0 values per item of the small-bank kernel (5 or 8)
};

// Tile-dependent fields of batch run r for `tile` (0-based, -1: direct).
// Returns the tile used: -1 when the run's window does not fit in LDS.
int assign_run_tile(BatchPlan &pl, int r, int tile, const ft_run &R, const double *f0h, const double *f1h,
                    double t_sft)
{
    EvalRun &E = pl.runs[r];
    if (tile >= 0 && tile_cfg(tile).L > 1 && !pl.uniform[r]) tile = 14;
    WindowPlan wp;
    if (tile >= 0) {
        wp = plan_window(f0h + R.f0_begin, R.n_f0, f1h + R.f1_begin, R.n_f1, pl.sky_tile.data() + 3 * pl.sky_prefix[r],
                         R.n_sky, pl.dt_absmax[r], pl.vmax[r], t_sft, tile);
        if (wp.tile < 0) tile = -1;  // window beyond the LDS budget: direct
    }
    E.wt = tile >= 0 ? wp.wt : 0;
    E.wtp = tile >= 0 ? wp.wtp : 0;
    E.tiles_f0 = tile >= 0 ? wp.tiles_f0 : 0;
    E.tiles_f1 = tile >= 0 ? wp.tiles_f1 : 0;
    E.tiles_sky = tile >= 0 ? wp.tiles_sky : 0;
    pl.tile[r] = tile;
    return tile;
}

// Work items of batch run r: its tiles, or for the small-bank kernel its
// (f0 chunk, 64-wide (f1, sky) chunk) pairs.
int64_t run_items(const BatchPlan &pl, int r)
{
    const EvalRun &E = pl.runs[r];
    if (pl.tile[r] >= 0) return (int64_t)E.tiles_f0 * E.tiles_f1 * E.tiles_sky;
    return (int64_t)((E.n_f0 + pl.small_chunk - 1) / pl.small_chunk) * (((int64_t)E.n_f1 * E.n_sky + 63) / 64);
}

// f0 chunk of the small-bank kernel for the batch's small runs: the one with
// fewer modelled lane operations, counting per item and SFT a fixed part
// (Doppler factor, f1 dt, loads: about 1.5 bins' worth) plus one bin, gather
// and add per f0 slot.  Label campaigns (5 f0 values per run) take 5; a batch
// of 16- or 24-value runs takes 8.
int choose_small_chunk(const BatchPlan &pl)
{
    double cost[2] = {0.0, 0.0};
    const int chunks[2] = {5, 8};
    for (size_t r = 0; r < pl.runs.size(); ++r) {
        if (pl.tile[r] >= 0) continue;
        const EvalRun &E = pl.runs[r];
        const double js = (double)(((int64_t)E.n_f1 * E.n_sky + 63) / 64) * (double)E.n_sft;
        for (int q = 0; q < 2; ++q)
            cost[q] += (double)((E.n_f0 + chunks[q] - 1) / chunks[q]) * js * (1.5 + chunks[q]);
    }
    return cost[0] < cost[1] ? 5 : 8;
}

void append_items(const BatchPlan &pl, int r, std::vector<int2> &out)
{
    const int64_t n = run_items(pl, r);
    for (int64_t t = 0; t < n; ++t) out.push_back(make_int2(r, (int)t));
}

// Size class of a batch run for the tile cache; -1 for f0 grids too small for
// a 64-wide f0 tile (the direct kernel evaluates them, one lane per template).
int batch_class(const ft_run &R, bool uniform)
{
    if (R.n_f0 < 32) return -1;
    const int b = std::min(floor_log2(R.n_f0) - 5, 7);
    const int j = std::min<int>(R.n_f1, 8) - 1;
    return (uniform ? 64 : 0) + b * 8 + j;
}

}  // namespace

static ft_status launch_batch_sequence(ft_ctx c, const BatchPlan &pl, bool generate, hipStream_t st)
{
    auto &b = c->bb;
    const int n_runs = (int)pl.runs.size();
    hipError_t e = launch_fill_u32(c->d_err, 0u, 1, st);
    if (e == hipSuccess) e = launch_fill_u32(b.counters, 0u, tile_count() + 1, st);
    if (e == hipSuccess)
        e = launch_batch_dt(b.tmid, b.sft_begin, b.tref, b.dt_prefix, n_runs, pl.dt_prefix[n_runs], b.dt, st);
    if (e == hipSuccess && generate)
        e = launch_gen_tables(b.gen, n_runs, b.gen_prefix, pl.gen_prefix_sft[n_runs], b.gen, n_runs,
                              b.gen_prefix, pl.gen_prefix_sft[n_runs], st);
    // the evaluation launches (one persistent launch per tile, then the
    // small-bank kernel) draw on disjoint work and run concurrently: the
    // first on st, the others on side streams forked from st and joined back
    // before the selection (a captured graph gets parallel branches), so one
    // launch's last workgroups overlap the next launch
    struct Launch {
        int id;  // tile, or tile_count() for the small-bank kernel
        int64_t off;
        int n;
    };
    std::vector<Launch> ls;
    int64_t item_off = 0;
    for (int id = 0; id <= tile_count(); ++id) {
        const int n_items = (int)pl.items[id].size();
        if (n_items > 0) ls.push_back({id, item_off, n_items});
        item_off += n_items;
    }
    const int n_side = std::min<int>((int)ls.size() - 1, ft_ctx_s::kSide);
    if (e == hipSuccess && n_side > 0) e = hipEventRecord(c->fork_ev, st);
    int joined = 0;  // side streams that waited on the fork (and must be joined back)
    for (int i = 0; i < n_side && e == hipSuccess; ++i) {
        e = hipStreamWaitEvent(c->side[i], c->fork_ev, 0);
        if (e == hipSuccess) joined = i + 1;
    }
    for (size_t i = 0; i < ls.size() && e == hipSuccess; ++i) {
        const Launch &L = ls[i];
        hipStream_t s = i == 0 || n_side == 0 ? st : c->side[(i - 1) % n_side];
        if (L.id < tile_count())
            e = launch_eval_batch(b.runs, b.items + L.off, L.n, pl.group_wtp[L.id], b.counters + L.id,
                                  std::min(L.n, 2048), tile_cfg(L.id), s);
        else
            e = launch_eval_batch_small(b.runs, b.items + L.off, L.n, pl.small_chunk, b.counters + tile_count(),
                                        std::min(L.n, 8192), s);
    }
    for (int i = 0; i < joined; ++i) {
        hipError_t ej = hipEventRecord(c->join_ev[i], c->side[i]);
        if (ej == hipSuccess) ej = hipStreamWaitEvent(st, c->join_ev[i], 0);
        if (e == hipSuccess) e = ej;
    }
    if (e == hipSuccess)
        e = launch_select_batch(b.runs, n_runs, c->batch_k, c->batch_cap, b.cand, b.s64, b.out, b.nout, b.maxz, c->d_err,
                                st);
    if (e != hipSuccess) return hip_fail(c, e, "launch batch");
    return FT_OK;
}

// Autotuning of batch size classes.  The base arrays must be on the device;
// the time offsets and tables are produced first.  Pass p launches the work
// items of every class with its p-th candidate tile, each class in a
// persistent launch of its own between two events, after one untimed pass
// that brings the clocks up.  The fastest tile of each class is cached.
static ft_status tune_batch(ft_ctx c, BatchPlan &pl, const std::vector<ft_run> &runs, const double *f0h,
                            const double *f1h, double t_sft, bool gen, const std::map<int, std::vector<int>> &classes)
{
    const auto t_start = std::chrono::steady_clock::now();
    auto &b = c->bb;
    const int n_runs = (int)pl.runs.size();
    hipError_t e = launch_batch_dt(b.tmid, b.sft_begin, b.tref, b.dt_prefix, n_runs, pl.dt_prefix[n_runs], b.dt, c->stream);
    if (e == hipSuccess && gen)
        e = launch_gen_tables(b.gen, n_runs, b.gen_prefix, pl.gen_prefix_sft[n_runs], b.gen, n_runs,
                              b.gen_prefix, pl.gen_prefix_sft[n_runs], c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "tile tuning");
    struct Cls {
        int id;
        std::vector<int> runs, cand;
        std::vector<double> rate;
        double evals;
    };
    std::vector<Cls> cls;
    size_t n_pass = 0;
    for (const auto &kv : classes) {
        Cls cl;
        cl.id = kv.first;
        cl.runs = kv.second;
        double w = 0.0, s0 = 0.0, s1 = 0.0;
        for (int r : cl.runs) {
            const ft_run &R = runs[r];
            const double ev = (double)R.n_f0 * R.n_f1 * R.n_sky * R.n_sft;
            w += ev;
            s0 += ev * R.n_f0;
            s1 += ev * R.n_f1;
        }
        cl.evals = w;
        cl.cand = tune_candidates(s0 / w, s1 / w, pl.uniform[cl.runs[0]] != 0);
        cl.rate.assign(cl.cand.size(), 0.0);
        n_pass = std::max(n_pass, cl.cand.size());
        cls.push_back(std::move(cl));
    }
    const size_t nc = cls.size();
    std::vector<hipEvent_t> ev(2 * nc, nullptr);
    ft_status st = FT_OK;
    for (auto &x : ev)
        if (hipEventCreate(&x) != hipSuccess) {
            x = nullptr;
            st = fail(c, FT_E_DEVICE, "hipEventCreate");
            break;
        }
    std::vector<int2> items;
    std::vector<size_t> off(nc + 1, 0);
    std::vector<char> active(nc, 0);
    std::vector<int> wtp(nc, 64);
    for (int pp = -1; pp < (int)n_pass && st == FT_OK; ++pp) {
        const size_t p = pp < 0 ? 0 : (size_t)pp;
        items.clear();
        for (size_t q = 0; q < nc; ++q) {
            off[q] = items.size();
            active[q] = p < cls[q].cand.size();
            wtp[q] = 64;
            if (!active[q]) continue;
            const int tile = cls[q].cand[p];
            int64_t n_items = 0;
            for (int r : cls[q].runs) {
                if (assign_run_tile(pl, r, tile, runs[r], f0h, f1h, t_sft) != tile) {
                    active[q] = 0;  // some run's window does not fit this tile
                    break;
                }
                wtp[q] = std::max(wtp[q], pl.runs[r].wtp);
                n_items += run_items(pl, r);
            }
            if (active[q] && (int64_t)items.size() + n_items >= 0x7fffffffLL) active[q] = 0;
            if (!active[q]) continue;
            for (int r : cls[q].runs) append_items(pl, r, items);
            // longest first, as the batch launch orders them
            std::stable_sort(items.begin() + (int64_t)off[q], items.end(), [&](const int2 &a, const int2 &b2) {
                return pl.runs[a.x].n_sft > pl.runs[b2.x].n_sft;
            });
        }
        off[nc] = items.size();
        if (items.empty()) continue;
        e = ensure(&b.items, &b.c_items, items.size());
        if (e == hipSuccess)
            e = hipMemcpyAsync(b.runs, pl.runs.data(), (size_t)n_runs * sizeof(EvalRun), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b.items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = launch_fill_u32(b.counters, 0u, (int)nc, c->stream);
        for (size_t q = 0; q < nc && e == hipSuccess; ++q) {
            if (!active[q]) continue;
            const int n_items = (int)(off[q + 1] - off[q]);
            e = hipEventRecord(ev[2 * q], c->stream);
            if (e == hipSuccess)
                e = launch_eval_batch(b.runs, b.items + off[q], n_items, wtp[q], b.counters + q, std::min(n_items, 2048),
                                      tile_cfg(cls[q].cand[p]), c->stream);
            if (e == hipSuccess) e = hipEventRecord(ev[2 * q + 1], c->stream);
        }
        // the host item list is reused by the next pass
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        for (size_t q = 0; q < nc && e == hipSuccess && pp >= 0; ++q) {
            if (!active[q]) continue;
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[2 * q], ev[2 * q + 1]);
            if (e == hipSuccess && ms > 0.f) cls[q].rate[p] = cls[q].evals / (ms * 1e-3);
        }
        if (e != hipSuccess) st = hip_fail(c, e, "tile tuning");
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (st != FT_OK) return st;
    c->tune_log.clear();
    for (const Cls &cl : cls) {
        size_t bi = 0;
        for (size_t i = 1; i < cl.cand.size(); ++i)
            if (cl.rate[i] > cl.rate[bi]) bi = i;
        if (cl.rate[bi] > 0.0) c->tune_cache[{1, (int64_t)cl.id}] = cl.cand[bi];
        for (size_t i = 0; i < cl.cand.size(); ++i) {
            ft_tune_entry t{};
            t.klass = 1 + cl.id;
            t.tile = cl.cand[i] + 1;
            t.chosen = cl.rate[bi] > 0.0 && i == bi;
            t.evals_per_s = cl.rate[i];
            t.sample_evals = cl.evals;
            c->tune_log.push_back(t);
        }
    }
    c->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return FT_OK;
}

ft_status ft_eval_batch(ft_ctx c, const ft_batch *bt, int32_t use_graph)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    if (!bt || bt->n_runs < 1 || !bt->runs) return fail(c, FT_E_INVALID, "batch needs n_runs >= 1 and runs");
    if (bt->k < 1 || bt->k > 512) return fail(c, FT_E_INVALID, "batch k must be in [1, 512]");
    if (bt->n_sft_total < 1 || !bt->t_mid || !bt->v_over_c) return fail(c, FT_E_INVALID, "batch SFT arrays missing");
    if (!(bt->t_sft > 0.0) || !is_finite(bt->t_sft)) return fail(c, FT_E_INVALID, "t_sft must be finite and > 0");
    if (bt->n_f0_total < 1 || bt->n_f1_total < 1 || bt->n_sky_total < 1 || !bt->f0 || !bt->f1 || !bt->sky_xyz)
        return fail(c, FT_E_INVALID, "batch bank arrays missing");
    if (bt->generate != 0 && bt->generate != 1) return fail(c, FT_E_INVALID, "generate must be 0 or 1");
    const bool gen = bt->generate == 1;
    if (gen && !bt->arms) return fail(c, FT_E_INVALID, "generated batches need arms");
    if (!gen && (!bt->power || bt->power_len < 1)) return fail(c, FT_E_INVALID, "batch tables missing");
    if (bt->tile < FT_TILE_TUNE || bt->tile > tile_count()) return fail(c, FT_E_INVALID, "unknown tile");
    const int n_runs = bt->n_runs;
    const int64_t NS = bt->n_sft_total;
    std::vector<ft_run> runs;
    std::vector<double> tm, vh, ah, f0h, f1h, skyh;
    if (fetch(runs, bt->runs, (size_t)n_runs) != hipSuccess || fetch(tm, bt->t_mid, (size_t)NS) != hipSuccess ||
        fetch(vh, bt->v_over_c, (size_t)NS * 3) != hipSuccess || (gen && fetch(ah, bt->arms, (size_t)NS * 6) != hipSuccess) ||
        fetch(f0h, bt->f0, (size_t)bt->n_f0_total) != hipSuccess || fetch(f1h, bt->f1, (size_t)bt->n_f1_total) != hipSuccess ||
        fetch(skyh, bt->sky_xyz, (size_t)bt->n_sky_total * 3) != hipSuccess)
        return fail(c, FT_E_INVALID, "cannot read the batch arrays");
    std::vector<double> vabs((size_t)NS);
    std::map<std::pair<int32_t, int32_t>, std::array<double, 3>> slice_extremes;  // (min t, max t, max |v|)
    for (int64_t k = 0; k < NS; ++k) {
        const double x = vh[3 * k], y = vh[3 * k + 1], z = vh[3 * k + 2];
        if (!is_finite(tm[k]) || !is_finite(x) || !is_finite(y) || !is_finite(z))
            return fail(c, FT_E_INVALID, "batch SFT arrays hold a non-finite value");
        vabs[k] = std::sqrt(x * x + y * y + z * z);
        if (!(vabs[k] < 1.0)) return fail(c, FT_E_INVALID, "|v|/c must be < 1");
    }
    for (double a : ah)
        if (!is_finite(a)) return fail(c, FT_E_INVALID, "arms hold a non-finite value");
    for (int64_t sk = 0; sk < bt->n_sky_total; ++sk) {
        const double x = skyh[3 * sk], y = skyh[3 * sk + 1], z = skyh[3 * sk + 2];
        if (!is_finite(x) || !is_finite(y) || !is_finite(z) || std::fabs(std::sqrt(x * x + y * y + z * z) - 1.0) > 1e-12)
            return fail(c, FT_E_INVALID, "batch sky vectors must be finite unit vectors");
    }
    for (double f : f1h)
        if (!is_finite(f)) return fail(c, FT_E_INVALID, "batch f1 must be finite");

    BatchPlan pl;
    pl.runs.resize(n_runs);
    pl.tile.resize(n_runs);
    pl.items.assign(tile_count() + 1, {});
    pl.dt_prefix.assign(n_runs + 1, 0);
    pl.stats_prefix.assign(n_runs + 1, 0);
    pl.gen_prefix_sft.assign(n_runs + 1, 0);
    pl.gen_prefix_elem.assign(n_runs + 1, 0);
    pl.sky_prefix.assign(n_runs + 1, 0);
    pl.sft_begin.resize(n_runs);
    pl.tref.resize(n_runs);
    pl.uniform.assign(n_runs, 0);
    pl.dt_absmax.assign(n_runs, 0.0);
    pl.vmax.assign(n_runs, 0.0);
    for (int r = 0; r < n_runs; ++r) {
        const ft_run &R = runs[r];
        if (R.n_sft < 1 || R.sft_begin < 0 || (int64_t)R.sft_begin + R.n_sft > NS)
            return fail(c, FT_E_INVALID, "run %d: SFT slice out of range", r);
        if (R.n_bins < 1 || R.first_bin < 0 || R.first_bin + (int64_t)R.n_bins >= 0x7fffffffLL)
            return fail(c, FT_E_INVALID, "run %d: bad table columns", r);
        if (R.n_bins >= (1 << 28))
            return fail(c, FT_E_UNSUPPORTED, "run %d: batch tables hold fewer than 2^28 columns", r);
        if (R.n_f0 < 1 || R.n_f1 < 1 || R.n_sky < 1 || R.f0_begin < 0 || R.f1_begin < 0 || R.sky_begin < 0 ||
            (int64_t)R.f0_begin + R.n_f0 > bt->n_f0_total || (int64_t)R.f1_begin + R.n_f1 > bt->n_f1_total ||
            (int64_t)R.sky_begin + R.n_sky > bt->n_sky_total)
            return fail(c, FT_E_INVALID, "run %d: bank slice out of range", r);
        if (!is_finite(R.t_ref)) return fail(c, FT_E_INVALID, "run %d: t_ref must be finite", r);
        const int64_t cells = (int64_t)R.n_sft * R.n_bins;
        if (!gen && (R.table_offset < 0 || R.table_offset + cells > bt->power_len))
            return fail(c, FT_E_INVALID, "run %d: table slice out of range", r);
        if (gen) {
            const char *msg = injection_error(R.inj);
            if (msg) return fail(c, FT_E_INVALID, "run %d: %s", r, msg);
        }
        const double *f0 = f0h.data() + R.f0_begin;
        const double *f1 = f1h.data() + R.f1_begin;
        for (int i = 0; i < R.n_f0; ++i)
            if (!is_finite(f0[i]) || !(f0[i] > 0.0) || (i > 0 && !(f0[i] > f0[i - 1])))
                return fail(c, FT_E_INVALID, "run %d: f0 must be finite, > 0 and strictly increasing", r);
        // extremes of the run's SFT slice, once per distinct slice (campaigns
        // often share one); t - t_ref rounds monotonically in t, so the
        // extreme time offsets are those of the extreme mid-times
        auto slice = slice_extremes.find({R.sft_begin, R.n_sft});
        if (slice == slice_extremes.end()) {
            std::array<double, 3> x{1e300, -1e300, 0.0};
            for (int k = R.sft_begin; k < R.sft_begin + R.n_sft; ++k) {
                x[0] = std::min(x[0], tm[k]);
                x[1] = std::max(x[1], tm[k]);
                x[2] = std::max(x[2], vabs[k]);
            }
            slice = slice_extremes.emplace(std::make_pair(R.sft_begin, R.n_sft), x).first;
        }
        const double dt_min = slice->second[0] - R.t_ref, dt_max = slice->second[1] - R.t_ref;
        const double vmax = slice->second[2];
        double f1_min = 1e300, f1_max = -1e300;
        for (int j = 0; j < R.n_f1; ++j) {
            f1_min = std::min(f1_min, f1[j]);
            f1_max = std::max(f1_max, f1[j]);
        }
        const double cs[4] = {f1_min * dt_min, f1_min * dt_max, f1_max * dt_min, f1_max * dt_max};
        const double c_min = *std::min_element(cs, cs + 4), c_max = *std::max_element(cs, cs + 4);
        if (!(f0[0] + c_min > 0.0)) return fail(c, FT_E_INVALID, "run %d: f0 + f1*(t - t_ref) must stay > 0", r);
        const double x_max = (f0[R.n_f0 - 1] + c_max) * (1.0 + vmax) * bt->t_sft;
        if (!(x_max < 2147483000.0)) return fail(c, FT_E_UNSUPPORTED, "run %d: frequencies above 2^31/T_sft", r);
        // sky order of the run
        std::vector<double> sky_run(skyh.begin() + 3 * (size_t)R.sky_begin, skyh.begin() + 3 * ((size_t)R.sky_begin + R.n_sky));
        std::vector<int32_t> perm;
        sky_order(sky_run, R.n_sky, perm);
        const size_t sky_base = pl.sky_tile.size() / 3;
        for (int sk = 0; sk < R.n_sky; ++sk) {
            for (int d = 0; d < 3; ++d) pl.sky_tile.push_back(sky_run[3 * (size_t)perm[sk] + d]);
            pl.perm.push_back(perm[sk]);
        }
        EvalRun &E = pl.runs[r];
        E = EvalRun{};
        guard_params(f0, R.n_f0, f0[R.n_f0 - 1], x_max, vmax, bt->t_sft, E.dT, E.eta);
        pl.uniform[r] = E.eta < 1e-4;
        pl.dt_absmax[r] = std::max(std::fabs(dt_min), std::fabs(dt_max));
        pl.vmax[r] = vmax;
        E.n_sft = R.n_sft;
        E.n_bins = R.n_bins;
        E.first_bin = (int32_t)R.first_bin;
        E.n_f0 = R.n_f0;
        E.n_f1 = R.n_f1;
        E.n_sky = R.n_sky;
        E.t_sft = bt->t_sft;
        E.sum_mode = FT_SUM_BLOCKED;
        pl.sft_begin[r] = R.sft_begin;
        pl.tref[r] = R.t_ref;
        pl.dt_prefix[r + 1] = pl.dt_prefix[r] + R.n_sft;
        pl.stats_prefix[r + 1] = pl.stats_prefix[r] + (int64_t)R.n_f0 * R.n_f1 * R.n_sky;
        pl.gen_prefix_sft[r + 1] = pl.gen_prefix_sft[r] + R.n_sft;
        pl.gen_prefix_elem[r + 1] = pl.gen_prefix_elem[r] + cells;
        pl.sky_prefix[r + 1] = pl.sky_prefix[r] + R.n_sky;
    }
    // Tile of every run: the forced one, the tile cached for its size class,
    // else the cost model; with FT_TILE_TUNE, uncached classes are timed below.
    std::map<int, std::vector<int>> to_tune;
    auto plan_tiles = [&]() {
        for (int r = 0; r < n_runs; ++r) {
            const ft_run &R = runs[r];
            const int kl = batch_class(R, pl.uniform[r] != 0);
            int tile;
            if (bt->tile > 0) {
                tile = bt->tile - 1;
            } else if (kl < 0) {
                tile = -1;
            } else {
                const auto it = c->tune_cache.find({1, (int64_t)kl});
                tile = it != c->tune_cache.end() ? it->second : choose_batch_tile(R.n_f0, R.n_f1, pl.uniform[r] != 0);
                if (it == c->tune_cache.end() && bt->tile == FT_TILE_TUNE) to_tune[kl].push_back(r);
            }
            assign_run_tile(pl, r, tile, R, f0h.data(), f1h.data(), bt->t_sft);
        }
    };
    plan_tiles();
    const int k = bt->k;
    const int cap = std::max(4096, 8 * k);

    // device buffers
    auto &b = c->bb;
    hipError_t e;
    const int64_t n_dt = pl.dt_prefix[n_runs], n_stats = pl.stats_prefix[n_runs];
    const int64_t n_power = gen ? pl.gen_prefix_elem[n_runs] : bt->power_len;
    if ((e = ensure(&b.tmid, &b.c_tmid, (size_t)NS)) != hipSuccess || (e = ensure(&b.v, &b.c_v, (size_t)NS * 3)) != hipSuccess ||
        (gen && (e = ensure(&b.arms, &b.c_arms, (size_t)NS * 6)) != hipSuccess) ||
        (e = ensure(&b.dt, &b.c_dt, (size_t)n_dt)) != hipSuccess ||
        (e = ensure(&b.f0, &b.c_f0, (size_t)bt->n_f0_total)) != hipSuccess ||
        (e = ensure(&b.f1, &b.c_f1, (size_t)bt->n_f1_total)) != hipSuccess ||
        (e = ensure(&b.sky, &b.c_sky, (size_t)bt->n_sky_total * 3)) != hipSuccess ||
        (e = ensure(&b.sky_tile, &b.c_sky_tile, pl.sky_tile.size())) != hipSuccess ||
        (e = ensure(&b.perm, &b.c_perm, pl.perm.size())) != hipSuccess ||
        (e = ensure(&b.tref, &b.c_tref, (size_t)n_runs)) != hipSuccess ||
        (e = ensure(&b.sft_begin, &b.c_sft_begin, (size_t)n_runs)) != hipSuccess ||
        (e = ensure(&b.dt_prefix, &b.c_dt_prefix, (size_t)n_runs + 1)) != hipSuccess ||
        (e = ensure(&b.power, &b.c_power, (size_t)n_power)) != hipSuccess ||
        (e = ensure(&b.stats, &b.c_stats, (size_t)n_stats)) != hipSuccess ||
        (e = ensure(&b.runs, &b.c_runs, (size_t)n_runs)) != hipSuccess ||
        (e = ensure(&b.counters, &b.c_counters, (size_t)std::max(tile_count() + 1, 129))) != hipSuccess ||
        (e = ensure(&b.cand, &b.c_cand, (size_t)n_runs * cap)) != hipSuccess ||
        (e = ensure(&b.s64, &b.c_s64, (size_t)n_runs * cap)) != hipSuccess ||
        (e = ensure(&b.out, &b.c_out, (size_t)n_runs * k)) != hipSuccess ||
        (e = ensure(&b.nout, &b.c_nout, (size_t)n_runs)) != hipSuccess ||
        (e = ensure(&b.maxz, &b.c_maxz, (size_t)n_runs)) != hipSuccess ||
        (e = ensure(&b.labels, &b.c_labels, (size_t)n_runs)) != hipSuccess ||
        (gen && ((e = ensure(&b.gen, &b.c_gen, (size_t)n_runs)) != hipSuccess ||
                 (e = ensure(&b.gen_prefix, &b.c_gen_prefix, (size_t)(n_runs + 1) * 2)) != hipSuccess ||
                 (e = ensure(&b.inj_bin, &b.c_inj_bin, (size_t)pl.gen_prefix_sft[n_runs])) != hipSuccess ||
                 (e = ensure(&b.inj_amp, &b.c_inj_amp, (size_t)pl.gen_prefix_sft[n_runs] * 3)) != hipSuccess ||
                 (e = ensure(&b.band, &b.c_band, (size_t)pl.gen_prefix_sft[n_runs] * 2)) != hipSuccess)))
        return hip_fail(c, e, "alloc batch buffers");
    // device pointers of every run
    for (int r = 0; r < n_runs; ++r) {
        const ft_run &R = runs[r];
        EvalRun &E = pl.runs[r];
        E.power = b.power + (gen ? pl.gen_prefix_elem[r] : R.table_offset);
        E.power_w = E.power;
        E.weight = nullptr;
        E.dt = b.dt + pl.dt_prefix[r];
        E.v = b.v + 3 * (int64_t)R.sft_begin;
        E.f0 = b.f0 + R.f0_begin;
        E.f1 = b.f1 + R.f1_begin;
        E.sky = b.sky + 3 * (int64_t)R.sky_begin;
        E.sky_tile = b.sky_tile + 3 * pl.sky_prefix[r];
        E.sky_perm = b.perm + pl.sky_prefix[r];
        E.stats = b.stats + pl.stats_prefix[r];
        E.err = c->d_err;
        if (gen) {
            GenRun g{};
            g.seed = R.seed;
            g.run = R.run_id;
            g.sft_offset = 0;
            g.n_sft = R.n_sft;
            g.n_bins = R.n_bins;
            g.first_bin = R.first_bin;
            g.t_mid = b.tmid + R.sft_begin;
            g.v = b.v + 3 * (int64_t)R.sft_begin;
            g.arms = b.arms + 6 * (int64_t)R.sft_begin;
            g.t_ref = R.t_ref;
            g.t_sft = bt->t_sft;
            g.amp = R.inj.amp;
            g.cos_iota = R.inj.cos_iota;
            g.psi = R.inj.psi;
            for (int d = 0; d < 3; ++d) g.sky[d] = R.inj.sky[d];
            g.f0 = R.inj.f0;
            g.f1 = R.inj.f1;
            g.ap = R.inj.ap;
            g.omega = R.inj.omega;
            g.phib = R.inj.phib;
            g.table = b.power + pl.gen_prefix_elem[r];
            g.inj_bin = b.inj_bin + pl.gen_prefix_sft[r];
            g.inj_amp = b.inj_amp + 3 * pl.gen_prefix_sft[r];
            g.n_inj = 1;
            g.band_mode = 1;
            g.n_bank_sky = R.n_sky;
            g.bank_sky = b.sky + 3 * (int64_t)R.sky_begin;
            const double *f0r = f0h.data() + R.f0_begin, *f1r = f1h.data() + R.f1_begin;
            g.bank_f0_lo = f0r[0];
            g.bank_f0_hi = f0r[R.n_f0 - 1];
            g.bank_f1_lo = *std::min_element(f1r, f1r + R.n_f1);
            g.bank_f1_hi = *std::max_element(f1r, f1r + R.n_f1);
            g.band = b.band + 2 * pl.gen_prefix_sft[r];
            pl.gen.push_back(g);
        }
    }
    std::vector<int64_t> gp;
    if (gen) {
        gp = pl.gen_prefix_sft;
        gp.insert(gp.end(), pl.gen_prefix_elem.begin(), pl.gen_prefix_elem.end());
    }
    struct Up {
        void *dst;
        const void *src;
        size_t bytes;
    } ups[] = {
        {b.tmid, tm.data(), tm.size() * 8},
        {b.v, vh.data(), vh.size() * 8},
        {b.arms, ah.data(), ah.size() * 8},
        {b.f0, f0h.data(), f0h.size() * 8},
        {b.f1, f1h.data(), f1h.size() * 8},
        {b.sky, skyh.data(), skyh.size() * 8},
        {b.sky_tile, pl.sky_tile.data(), pl.sky_tile.size() * 8},
        {b.perm, pl.perm.data(), pl.perm.size() * 4},
        {b.tref, pl.tref.data(), pl.tref.size() * 8},
        {b.sft_begin, pl.sft_begin.data(), pl.sft_begin.size() * 4},
        {b.dt_prefix, pl.dt_prefix.data(), pl.dt_prefix.size() * 8},
        {b.gen, pl.gen.data(), pl.gen.size() * sizeof(GenRun)},
        {b.gen_prefix, gp.data(), gp.size() * 8},
    };
    for (const Up &u : ups) {
        if (u.bytes == 0 || !u.dst) continue;
        e = hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "upload batch");
    }
    if (!gen) {
        e = hipMemcpyAsync(b.power, bt->power, (size_t)bt->power_len * sizeof(float), hipMemcpyDefault, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "upload batch tables");
    }
    if (!to_tune.empty()) {
        ft_status st = tune_batch(c, pl, runs, f0h.data(), f1h.data(), bt->t_sft, gen, to_tune);
        if (st != FT_OK) return st;
        to_tune.clear();
        plan_tiles();
    }
    // work items grouped by tile (the direct kernel's last)
    pl.small_chunk = choose_small_chunk(pl);
    int64_t total_items = 0;
    for (int r = 0; r < n_runs; ++r) total_items += run_items(pl, r);
    if (total_items >= 0x7fffffff) return fail(c, FT_E_UNSUPPORTED, "too many work items");
    pl.group_wtp.assign(tile_count() + 1, 64);
    for (int r = 0; r < n_runs; ++r) {
        const int t = pl.tile[r];
        append_items(pl, r, pl.items[t >= 0 ? t : tile_count()]);
        if (t >= 0) pl.group_wtp[t] = std::max(pl.group_wtp[t], pl.runs[r].wtp);
    }
    // longest first within each group (an item's time grows with its run's
    // SFT count): the workgroups draining a queue then end together, instead
    // of a few long items that were queued last running on an idle GPU
    for (auto &v : pl.items)
        std::stable_sort(v.begin(), v.end(), [&](const int2 &a, const int2 &b2) {
            return pl.runs[a.x].n_sft > pl.runs[b2.x].n_sft;
        });
    std::vector<int2> items_flat;
    items_flat.reserve((size_t)total_items);
    for (auto &v : pl.items) items_flat.insert(items_flat.end(), v.begin(), v.end());
    if ((e = ensure(&b.items, &b.c_items, (size_t)std::max<int64_t>(total_items, 1))) != hipSuccess)
        return hip_fail(c, e, "alloc batch items");
    e = hipMemcpyAsync(b.runs, pl.runs.data(), pl.runs.size() * sizeof(EvalRun), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.items, items_flat.data(), items_flat.size() * sizeof(int2), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "upload batch items");
    // the host vectors above are released on return: make the copies complete
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "upload batch");
    c->batch_runs = n_runs;
    c->batch_k = k;
    c->batch_cap = cap;
    c->have_batch = false;
    if (c->graph_exec) {
        (void)hipGraphExecDestroy(c->graph_exec);
        c->graph_exec = nullptr;
    }
    if (c->graph) {
        (void)hipGraphDestroy(c->graph);
        c->graph = nullptr;
    }
    if (use_graph) {
        if (!c->capture_stream && hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess)
            return fail(c, FT_E_DEVICE, "capture stream");
        e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(c, e, "begin capture");
        ft_status st = launch_batch_sequence(c, pl, gen, c->capture_stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->capture_stream, &g);
        if (st != FT_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e2 != hipSuccess) return hip_fail(c, e2, "end capture");
        c->graph = g;
        e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) return hip_fail(c, e, "instantiate graph");
        e = hipEventRecord(c->bev[0], c->stream);
        if (e == hipSuccess) e = hipGraphLaunch(c->graph_exec, c->stream);
        if (e == hipSuccess) e = hipEventRecord(c->bev[1], c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "launch graph");
    } else {
        e = hipEventRecord(c->bev[0], c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "record event");
        ft_status st = launch_batch_sequence(c, pl, gen, c->stream);
        if (st != FT_OK) return st;
        e = hipEventRecord(c->bev[1], c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "record event");
    }
    c->have_batch = true;
    return FT_OK;
}

ft_status ft_batch_replay(ft_ctx c)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (!c->have_batch || !c->graph_exec) return fail(c, FT_E_STATE, "no captured batch to replay");
    hipError_t e = hipEventRecord(c->bev[0], c->stream);
    if (e == hipSuccess) e = hipGraphLaunch(c->graph_exec, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->bev[1], c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "replay graph");
    return FT_OK;
}

ft_status ft_batch_toplist(ft_ctx c, int32_t run, ft_candidate *out, int32_t *n_out)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (!c->have_batch) return fail(c, FT_E_STATE, "no batch evaluated");
    if (run < 0 || run >= c->batch_runs) return fail(c, FT_E_INVALID, "run %d out of range", run);
    if (!out || !n_out) return fail(c, FT_E_INVALID, "out and n_out must be non-null");
    ft_status st = sync_and_check(c);
    if (st != FT_OK) return st;
    uint32_t flags = 0;
    if (hipMemcpy(&flags, c->d_err, sizeof flags, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, FT_E_DEVICE, "read flags");
    if (flags & ERR_CAND_OVERFLOW)
        return fail(c, FT_E_UNSUPPORTED, "a run has more tied toplist candidates than the batch buffer holds");
    int32_t n = 0;
    hipError_t e = hipMemcpy(&n, c->bb.nout + run, sizeof n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && n > 0)
        e = hipMemcpy(out, c->bb.out + (size_t)run * c->batch_k, (size_t)n * sizeof(ft_candidate), hipMemcpyDefault);
    if (e != hipSuccess) return hip_fail(c, e, "copy batch toplist");
    *n_out = n;
    return FT_OK;
}

ft_status ft_batch_labels(ft_ctx c, double tau, uint8_t *labels, double *max_z)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (!c->have_batch) return fail(c, FT_E_STATE, "no batch evaluated");
    if (!is_finite(tau)) return fail(c, FT_E_INVALID, "tau must be finite");
    hipError_t e = launch_labels(c->bb.maxz, c->batch_runs, tau, c->bb.labels, c->stream);
    if (e == hipSuccess && labels)
        e = hipMemcpyAsync(labels, c->bb.labels, (size_t)c->batch_runs, hipMemcpyDefault, c->stream);
    if (e == hipSuccess && max_z)
        e = hipMemcpyAsync(max_z, c->bb.maxz, (size_t)c->batch_runs * sizeof(double), hipMemcpyDefault, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "labels");
    ft_status st = sync_and_check(c);
    if (st != FT_OK) return st;
    uint32_t flags = 0;
    if (hipMemcpy(&flags, c->d_err, sizeof flags, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, FT_E_DEVICE, "read flags");
    if (flags & ERR_CAND_OVERFLOW)
        return fail(c, FT_E_UNSUPPORTED, "a run has more tied toplist candidates than the batch buffer holds");
    return FT_OK;
}

ft_status ft_batch_time(ft_ctx c, double *ms)
{
    if (!c || !ms) return FT_E_INVALID;
    if (!c->have_batch) return fail(c, FT_E_STATE, "no batch evaluated");
    ft_status st = sync_and_check(c);
    if (st != FT_OK) return st;
    float f = 0.f;
    if (hipEventElapsedTime(&f, c->bev[0], c->bev[1]) != hipSuccess) return fail(c, FT_E_DEVICE, "event time");
    *ms = f;
    return FT_OK;
}

// ---------------------------------------------------------------------------
// Surrogate MLP
// ---------------------------------------------------------------------------
struct ft_mlp_s {
    ft_ctx ctx = nullptr;
    MlpBufs m{};
    MlpConst cst{};
    int step = 0;
    float *d_raw = nullptr;
    size_t cap_raw = 0;
    float *d_y = nullptr;
    size_t cap_y = 0;
    float *d_prob = nullptr;
    size_t cap_prob = 0;
    std::vector<void *> allocs;
};

static void mlp_free(ft_mlp p)
{
    for (void *a : p->allocs) (void)hipFree(a);
    p->allocs.clear();
    release(&p->d_raw, &p->cap_raw);
    release(&p->d_y, &p->cap_y);
    release(&p->d_prob, &p->cap_prob);
}

}  // extern "C"

template <typename T>
static hipError_t mlp_alloc(ft_mlp p, T **dst, size_t n)
{
    size_t cap = 0;
    *dst = nullptr;
    hipError_t e = ensure(dst, &cap, n);
    if (e == hipSuccess) p->allocs.push_back((void *)*dst);
    return e;
}

extern "C" {

ft_status ft_mlp_create(ft_ctx c, const float *params, uint64_t seed, const float *feat_shift,
                        const float *feat_scale, int32_t max_batch, ft_mlp *out)
{
    if (!c || !out) return FT_E_INVALID;
    *out = nullptr;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    if (!feat_shift || !feat_scale || max_batch < 1) return fail(c, FT_E_INVALID, "feature map and max_batch >= 1 required");
    std::vector<float> sh, sc;
    if (fetch(sh, feat_shift, 6) != hipSuccess || fetch(sc, feat_scale, 6) != hipSuccess)
        return fail(c, FT_E_INVALID, "cannot read the feature map");
    for (int i = 0; i < 6; ++i)
        if (!is_finite(sh[i]) || !is_finite(sc[i]) || !(sc[i] != 0.0f)) return fail(c, FT_E_INVALID, "feature map must be finite, scale != 0");
    ft_mlp p = new ft_mlp_s();
    p->ctx = c;
    for (int i = 0; i < 6; ++i) {
        p->cst.shift[i] = sh[i];
        p->cst.scale[i] = sc[i];
    }
    const int mb = (max_batch + 63) / 64 * 64;
    p->m.max_batch = mb;
    const size_t act = (size_t)mb * MLP_H;
    MlpBufs &m = p->m;
    hipError_t e = hipSuccess;
    float **f32s[] = {&m.theta, &m.m, &m.v, &m.grad};
    for (float **q : f32s)
        if (e == hipSuccess) e = mlp_alloc(p, q, (size_t)MLP_N_PARAMS);
    if (e == hipSuccess) e = mlp_alloc(p, &m.w2b, (size_t)MLP_H * MLP_H);
    if (e == hipSuccess) e = mlp_alloc(p, &m.w3b, (size_t)MLP_H * MLP_H);
    if (e == hipSuccess) e = mlp_alloc(p, &m.w2t, (size_t)MLP_H * MLP_H);
    if (e == hipSuccess) e = mlp_alloc(p, &m.w3t, (size_t)MLP_H * MLP_H);
    float **acts[] = {&m.z1, &m.z2, &m.z3, &m.dz1, &m.dz2, &m.dz3};
    for (float **q : acts)
        if (e == hipSuccess) e = mlp_alloc(p, q, act);
    __bf16 **bacts[] = {&m.a1, &m.a2, &m.a3, &m.dz1b, &m.dz2b, &m.dz3b};
    for (__bf16 **q : bacts)
        if (e == hipSuccess) e = mlp_alloc(p, q, act);
    if (e == hipSuccess) e = mlp_alloc(p, &m.x, (size_t)mb * 6);
    if (e == hipSuccess) e = mlp_alloc(p, &m.logit, (size_t)mb);
    if (e == hipSuccess) e = mlp_alloc(p, &m.dlogit, (size_t)mb);
    if (e == hipSuccess) e = mlp_alloc(p, &m.loss, (size_t)1);
    if (e == hipSuccess) e = mlp_alloc(p, &m.lossv, (size_t)mb);
    if (e == hipSuccess) e = mlp_alloc(p, &m.part, (size_t)(mb / MLP_RED_ROWS + 1) * MLP_RED_VEC);
    if (e == hipSuccess) e = mlp_alloc(p, &m.wpart, (size_t)2 * MLP_MAX_SLICES * MLP_H * MLP_H);
    if (e != hipSuccess) {
        mlp_free(p);
        delete p;
        return hip_fail(c, e, "alloc MLP");
    }
    std::vector<float> theta((size_t)MLP_N_PARAMS, 0.0f);
    if (params) {
        if (hipMemcpy(theta.data(), params, theta.size() * 4, hipMemcpyDefault) != hipSuccess) {
            mlp_free(p);
            delete p;
            return fail(c, FT_E_INVALID, "cannot read params");
        }
        for (float x : theta)
            if (!is_finite(x)) {
                mlp_free(p);
                delete p;
                return fail(c, FT_E_INVALID, "params must be finite");
            }
    } else {  // He initialisation: N(0, 2/fan_in) weights, zero biases
        std::mt19937_64 rng(seed);
        const int fan[4] = {6, MLP_H, MLP_H, MLP_H};
        const int off[4] = {0, MLP_OFF_W2, MLP_OFF_W3, MLP_OFF_W4};
        const int cnt[4] = {MLP_H * 6, MLP_H * MLP_H, MLP_H * MLP_H, MLP_H};
        for (int l = 0; l < 4; ++l) {
            std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / fan[l]));
            for (int i = 0; i < cnt[l]; ++i) theta[(size_t)off[l] + i] = (float)nd(rng);
        }
    }
    std::vector<float> zeros((size_t)MLP_N_PARAMS, 0.0f);
    e = hipMemcpyAsync(m.theta, theta.data(), theta.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(m.m, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(m.v, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = mlp_refresh_bf16(m, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        mlp_free(p);
        delete p;
        return hip_fail(c, e, "init MLP");
    }
    *out = p;
    return FT_OK;
}

void ft_mlp_destroy(ft_mlp p)
{
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    (void)hipStreamSynchronize(p->ctx->stream);
    mlp_free(p);
    delete p;
}

ft_status ft_mlp_get_params(ft_mlp p, float *params)
{
    if (!p || !params) return FT_E_INVALID;
    ft_ctx c = p->ctx;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(params, p->m.theta, (size_t)MLP_N_PARAMS * 4, hipMemcpyDefault);
    if (e != hipSuccess) return hip_fail(c, e, "get params");
    return FT_OK;
}

static ft_status mlp_upload(ft_mlp p, const float *raw, const float *y, int64_t n)
{
    ft_ctx c = p->ctx;
    hipError_t e = ensure(&p->d_raw, &p->cap_raw, (size_t)n * 6);
    if (e == hipSuccess && y) e = ensure(&p->d_y, &p->cap_y, (size_t)n);
    if (e == hipSuccess) e = hipMemcpyAsync(p->d_raw, raw, (size_t)n * 6 * 4, hipMemcpyDefault, c->stream);
    if (e == hipSuccess && y) e = hipMemcpyAsync(p->d_y, y, (size_t)n * 4, hipMemcpyDefault, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "upload MLP data");
    // validate on the host (amp > 0 for the log feature, finite values, labels in [0, 1])
    std::vector<float> h;
    if (fetch(h, raw, (size_t)n * 6) != hipSuccess) return fail(c, FT_E_INVALID, "cannot read inputs");
    for (int64_t i = 0; i < n; ++i) {
        if (!(h[(size_t)i * 6] > 0.0f)) return fail(c, FT_E_INVALID, "input %lld: amplitude must be > 0", (long long)i);
        for (int j = 0; j < 6; ++j)
            if (!is_finite(h[(size_t)i * 6 + j])) return fail(c, FT_E_INVALID, "inputs must be finite");
    }
    if (y) {
        std::vector<float> hy;
        if (fetch(hy, y, (size_t)n) != hipSuccess) return fail(c, FT_E_INVALID, "cannot read labels");
        for (float v : hy)
            if (!(v >= 0.0f && v <= 1.0f)) return fail(c, FT_E_INVALID, "labels must lie in [0, 1]");
    }
    return FT_OK;
}

ft_status ft_mlp_predict(ft_mlp p, const float *raw, int64_t n, float *prob)
{
    if (!p) return FT_E_INVALID;
    ft_ctx c = p->ctx;
    c->err.clear();
    if (!raw || !prob || n < 1 || n > 0x7fffffff) return fail(c, FT_E_INVALID, "predict needs 1 <= n < 2^31 and buffers");
    ft_status st = mlp_upload(p, raw, nullptr, n);
    if (st != FT_OK) return st;
    hipError_t e = ensure(&p->d_prob, &p->cap_prob, (size_t)n);
    for (int64_t b0 = 0; b0 < n && e == hipSuccess; b0 += p->m.max_batch) {
        const int bsz = (int)std::min<int64_t>(p->m.max_batch, n - b0);
        MlpConst cst = p->cst;
        cst.base = b0;
        cst.n_total = n;
        cst.perm_a = 0;
        e = mlp_forward(p->m, p->d_raw, nullptr, cst, bsz, p->d_prob + b0, c->stream);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(prob, p->d_prob, (size_t)n * 4, hipMemcpyDefault, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "predict");
    return FT_OK;
}

ft_status ft_mlp_loss_grad(ft_mlp p, const float *raw, const float *y, int32_t n, float *loss, float *grad)
{
    if (!p) return FT_E_INVALID;
    ft_ctx c = p->ctx;
    c->err.clear();
    if (!raw || !y || !loss || !grad || n < 1 || n > p->m.max_batch)
        return fail(c, FT_E_INVALID, "loss_grad needs 1 <= n <= max_batch and buffers");
    ft_status st = mlp_upload(p, raw, y, n);
    if (st != FT_OK) return st;
    MlpConst cst = p->cst;
    cst.base = 0;
    cst.n_total = n;
    cst.perm_a = 0;
    hipError_t e = launch_fill_u32((uint32_t *)p->m.loss, 0u, 1, c->stream);
    if (e == hipSuccess) e = mlp_forward(p->m, p->d_raw, p->d_y, cst, n, nullptr, c->stream);
    if (e == hipSuccess) e = mlp_backward(p->m, n, nullptr, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(loss, p->m.loss, 4, hipMemcpyDefault, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(grad, p->m.grad, (size_t)MLP_N_PARAMS * 4, hipMemcpyDefault, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "loss_grad");
    return FT_OK;
}

ft_status ft_mlp_train(ft_mlp p, const float *raw, const float *y, int64_t n, int32_t batch, int32_t epochs,
                       float lr, uint64_t seed, float *epoch_loss)
{
    if (!p) return FT_E_INVALID;
    ft_ctx c = p->ctx;
    c->err.clear();
    if (!raw || !y || n < 1 || n > 0x7fffffff || batch < 1 || batch > p->m.max_batch || epochs < 0 ||
        !(lr > 0.0f) || !is_finite(lr))
        return fail(c, FT_E_INVALID, "train needs 1 <= batch <= max_batch, epochs >= 0, lr > 0");
    ft_status st = mlp_upload(p, raw, y, n);
    if (st != FT_OK) return st;
    std::mt19937_64 rng(seed);
    hipError_t e = hipSuccess;
    for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
        // affine permutation i -> (a i + b) mod n with gcd(a, n) = 1
        uint64_t a = 1 + rng() % (uint64_t)std::max<int64_t>(n - 1, 1);
        while (std::gcd(a, (uint64_t)n) != 1) a = a % (uint64_t)n + 1;
        const uint64_t b = rng() % (uint64_t)n;
        e = launch_fill_u32((uint32_t *)p->m.loss, 0u, 1, c->stream);
        int n_batches = 0;
        for (int64_t b0 = 0; b0 < n && e == hipSuccess; b0 += batch) {
            const int bsz = (int)std::min<int64_t>(batch, n - b0);
            MlpConst cst = p->cst;
            cst.base = b0;
            cst.n_total = n;
            cst.perm_a = n > 1 ? a : 0;
            cst.perm_c = b;
            e = mlp_forward(p->m, p->d_raw, p->d_y, cst, bsz, nullptr, c->stream);
            const MlpAdamStep adam{lr, ++p->step};
            if (e == hipSuccess) e = mlp_backward(p->m, bsz, &adam, c->stream);
            ++n_batches;
        }
        if (epoch_loss && e == hipSuccess) {
            float l = 0.0f;
            e = hipMemcpyAsync(&l, p->m.loss, 4, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            epoch_loss[ep] = l / (float)std::max(n_batches, 1);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "train");
    return FT_OK;
}

}  // extern "C"
