// Host layer of libfasttracks: argument validation, device buffers, tiling
// decisions and the stream-ordered launch sequence behind the C ABI of
// include/fasttracks.h.  No arithmetic of the statistic happens here; the host
// only derives launch parameters (window widths, guard margins) from bounds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
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
    double vmax = 0.0;
    float *d_power = nullptr;
    size_t cap_power = 0;
    float *d_weight = nullptr;
    size_t cap_weight = 0;
    float *d_power_w = nullptr;
    size_t cap_power_w = 0;
    double *d_tmid = nullptr, *d_v = nullptr, *d_dt = nullptr;
    size_t cap_tmid = 0, cap_v = 0, cap_dt = 0;
    double *d_mu_sigma = nullptr;
    uint32_t *d_err = nullptr;

    // bank
    std::vector<double> f0_h, f1_h, sky_h, sky_tile_h;
    std::vector<int32_t> perm_h;
    double *d_f0 = nullptr, *d_f1 = nullptr, *d_sky = nullptr, *d_edges = nullptr,
           *d_sky_tile = nullptr;
    size_t cap_f0 = 0, cap_f1 = 0, cap_sky = 0, cap_edges = 0, cap_sky_tile = 0;
    int32_t *d_perm = nullptr;
    size_t cap_perm = 0;
    float *d_stats = nullptr;
    size_t cap_stats = 0;

    // selection
    uint32_t *d_hist = nullptr, *d_state = nullptr, *d_cnt = nullptr, *d_off = nullptr,
             *d_fill = nullptr;
    size_t cap_hist = 0, cap_state = 0, cap_cnt = 0, cap_off = 0, cap_fill = 0;
    int64_t *d_cand = nullptr;
    double *d_cand_s64 = nullptr;
    size_t cap_cand = 0, cap_cand_s64 = 0;
    int32_t *d_seg = nullptr;
    size_t cap_seg = 0;
    ft_candidate *d_out = nullptr;
    size_t cap_out = 0;
    int32_t *d_nout = nullptr;
    size_t cap_nout = 0;
    unsigned long long *d_count = nullptr;
    int32_t *d_bins = nullptr;
    size_t cap_bins = 0;

    // last evaluation
    bool have_eval = false;
    EvalRun last_run{};
    bool last_grid = true;
    int last_k = 0, last_nsub = 0;
    int64_t last_cap = 0;
    double last_rel_err = 0.0;
    int last_tile = -1;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
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

int choose_tile(int64_t n_f0, int64_t n_f1, bool uniform)
{
    if (!uniform || n_f0 < 96) return n_f1 >= 4 ? 1 : 0;
    // prefer the run length and f1 tile that waste the fewest lanes
    const int cands[] = {3, 4, 5, 2, 7, 6};
    double best = 1e30;
    int best_id = 3;
    for (int id : cands) {
        const TileCfg &t = tile_cfg(id);
        const double f0w = std::ceil((double)n_f0 / (64.0 * t.L)) * 64.0 * t.L / (double)n_f0;
        const double f1w = std::ceil((double)n_f1 / t.JT) * t.JT / (double)n_f1;
        const double ops = (9.0 + t.L) / t.L;  // VALU per evaluation of the run loop
        const double cost = f0w * f1w * ops;
        if (cost < best - 1e-9) {
            best = cost;
            best_id = id;
        }
    }
    return best_id;
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
        hipMalloc(&c->d_count, sizeof(unsigned long long)) != hipSuccess) {
        ft_destroy(c);
        return FT_E_NOMEM;
    }
    (void)hipMemset(c->d_err, 0, sizeof(uint32_t));
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) {
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
    release(&c->d_tmid, &c->cap_tmid);
    release(&c->d_v, &c->cap_v);
    release(&c->d_dt, &c->cap_dt);
    release(&c->d_mu_sigma, nullptr);
    release(&c->d_err, nullptr);
    release(&c->d_f0, &c->cap_f0);
    release(&c->d_f1, &c->cap_f1);
    release(&c->d_sky, &c->cap_sky);
    release(&c->d_sky_tile, &c->cap_sky_tile);
    release(&c->d_perm, &c->cap_perm);
    release(&c->d_edges, &c->cap_edges);
    release(&c->d_stats, &c->cap_stats);
    release(&c->d_hist, &c->cap_hist);
    release(&c->d_state, &c->cap_state);
    release(&c->d_cnt, &c->cap_cnt);
    release(&c->d_off, &c->cap_off);
    release(&c->d_fill, &c->cap_fill);
    release(&c->d_cand, &c->cap_cand);
    release(&c->d_cand_s64, &c->cap_cand_s64);
    release(&c->d_seg, &c->cap_seg);
    release(&c->d_out, &c->cap_out);
    release(&c->d_nout, &c->cap_nout);
    release(&c->d_count, nullptr);
    release(&c->d_bins, &c->cap_bins);
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
    if ((e = launch_noise_moments(weight ? c->d_weight : nullptr, (int)total, c->d_mu_sigma,
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
    if (c->have_sfts && c->n_sft != (int32_t)total) c->have_vel = false;
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

ft_status ft_set_velocities(ft_ctx c, const double *v)
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
    if (e != hipSuccess) return hip_fail(c, e, "alloc velocities");
    e = hipMemcpyAsync(c->d_v, vh.data(), n3 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy velocities");
    c->vmax = vmax;
    c->have_vel = true;
    c->have_eval = false;
    return FT_OK;
}

static ft_status prepare_bank(ft_ctx c, const ft_bank *bank, double t_ref, EvalRun &run,
                              bool &grid, int64_t &n_t)
{
    if (!bank) return fail(c, FT_E_INVALID, "bank is null");
    if (!c->have_sfts || !c->have_vel) return fail(c, FT_E_STATE, "ft_set_sfts and ft_set_velocities must come first");
    if (!is_finite(t_ref)) return fail(c, FT_E_INVALID, "t_ref must be finite");
    grid = bank->kind == FT_BANK_GRID;
    if (!grid && bank->kind != FT_BANK_LIST) return fail(c, FT_E_INVALID, "unknown bank kind %d", bank->kind);
    if (!bank->f0 || !bank->f1 || !bank->sky_xyz) return fail(c, FT_E_INVALID, "bank arrays must be non-null");
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
    if (fetch(c->f0_h, bank->f0, (size_t)n0) != hipSuccess || fetch(c->f1_h, bank->f1, (size_t)n1) != hipSuccess ||
        fetch(c->sky_h, bank->sky_xyz, (size_t)ns * 3) != hipSuccess)
        return fail(c, FT_E_INVALID, "cannot read the bank arrays");
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
    const double x_max = (f0_max + c_max) * (1.0 + c->vmax) * c->t_sft;
    if (!(x_max < 2147483000.0)) return fail(c, FT_E_UNSUPPORTED, "track frequencies above 2^31/T_sft");

    // upload
    if ((e = ensure(&c->d_f0, &c->cap_f0, (size_t)n0)) != hipSuccess ||
        (e = ensure(&c->d_f1, &c->cap_f1, (size_t)n1)) != hipSuccess ||
        (e = ensure(&c->d_sky, &c->cap_sky, (size_t)ns * 3)) != hipSuccess ||
        (e = ensure(&c->d_stats, &c->cap_stats, (size_t)n_t)) != hipSuccess)
        return hip_fail(c, e, "alloc bank");
    if (grid) {
        sky_order(c->sky_h, ns, c->perm_h);
        c->sky_tile_h.resize((size_t)ns * 3);
        for (int64_t s = 0; s < ns; ++s)
            for (int d = 0; d < 3; ++d) c->sky_tile_h[3 * s + d] = c->sky_h[3 * (size_t)c->perm_h[s] + d];
        if ((e = ensure(&c->d_sky_tile, &c->cap_sky_tile, (size_t)ns * 3)) != hipSuccess ||
            (e = ensure(&c->d_perm, &c->cap_perm, (size_t)ns)) != hipSuccess)
            return hip_fail(c, e, "alloc sky order");
        e = hipMemcpyAsync(c->d_sky_tile, c->sky_tile_h.data(), ns * 3 * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->d_perm, c->perm_h.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "upload sky order");
    }
    e = hipMemcpyAsync(c->d_f0, c->f0_h.data(), n0 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_f1, c->f1_h.data(), n1 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_sky, c->sky_h.data(), ns * 3 * sizeof(double), hipMemcpyHostToDevice, c->stream);
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
    // bounds used by the grid kernel
    if (grid) {
        const double T = c->t_sft;
        double dT = n0 > 1 ? (c->f0_h[n0 - 1] - c->f0_h[0]) / (double)(n0 - 1) * T : T;
        double tau = 0.0;
        for (int64_t i = 0; i < n0; ++i)
            tau = std::max(tau, std::fabs(c->f0_h[i] - c->f0_h[0] - (double)i * (dT / T)));
        tau += 8.0 * std::ldexp(f0_max, -52);
        // eta bounds, in bins: the rounding of the canonical x + 1/2 and of the
        // estimate (f0 + c + 1/(2 g T)) * (g T) (each below 6 * 2^-53 * x_max),
        // the grid's deviation tau from uniform spacing, and the rounding of the
        // per-SFT drift e = dT*g - 1 over a run; doubled for margin.
        const double rho = 6.0 * std::ldexp(x_max, -53);
        double eta = 2.0 * (2.0 * rho + 2.0 * tau * (1.0 + c->vmax) * T + std::ldexp(1.0, -40));
        run.dT = dT;
        run.eta = eta;
        (void)dt_min;
    }
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
        (e = ensure(&c->d_seg, &c->cap_seg, (size_t)n_seg_map)) != hipSuccess ||
        (e = ensure(&c->d_out, &c->cap_out, (size_t)n_seg * k)) != hipSuccess ||
        (e = ensure(&c->d_nout, &c->cap_nout, (size_t)n_seg)) != hipSuccess)
        return hip_fail(c, e, "alloc selection buffers");
    return FT_OK;
}

static SelectBufs select_bufs(ft_ctx c, int64_t cap)
{
    SelectBufs b;
    b.hist = c->d_hist;
    b.state = c->d_state;
    b.cnt = c->d_cnt;
    b.off = c->d_off;
    b.fill = c->d_fill;
    b.cand = c->d_cand;
    b.cand_s64 = c->d_cand_s64;
    b.seg_of_f0 = c->d_seg;
    b.out = c->d_out;
    b.n_out = c->d_nout;
    b.mu_sigma = c->d_mu_sigma;
    b.cap = cap;
    return b;
}

ft_status ft_eval_templates(ft_ctx c, const ft_bank *bank, double t_ref, const ft_eval_opts *opts,
                            float *stats)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    if (!opts) return fail(c, FT_E_INVALID, "opts is null");
    if (opts->precision != FT_INDEX_FP64)
        return fail(c, FT_E_UNSUPPORTED,
                    "ft_eval_templates computes canonical FP64 bins; the FP32/df64/guarded index "
                    "forms are available through ft_count_index_mismatches and ft_bins");
    if (opts->k < 1 || opts->k > 65536) return fail(c, FT_E_INVALID, "k must be in [1, 65536]");
    if (opts->n_sub < 1 || opts->n_sub > 4096) return fail(c, FT_E_INVALID, "n_sub must be in [1, 4096]");
    if (!opts->sub_edges) return fail(c, FT_E_INVALID, "sub_edges is null");
    if (opts->sum_mode != FT_SUM_BLOCKED && opts->sum_mode != FT_SUM_PLAIN_FP32)
        return fail(c, FT_E_INVALID, "unknown sum_mode");
    std::vector<double> edges;
    if (fetch(edges, opts->sub_edges, (size_t)opts->n_sub + 1) != hipSuccess)
        return fail(c, FT_E_INVALID, "cannot read sub_edges");
    for (size_t j = 0; j < edges.size(); ++j) {
        if (!is_finite(edges[j])) return fail(c, FT_E_INVALID, "sub_edges must be finite");
        if (j > 0 && !(edges[j] > edges[j - 1])) return fail(c, FT_E_INVALID, "sub_edges must be strictly increasing");
    }
    EvalRun run;
    bool grid;
    int64_t n_t;
    ft_status st = prepare_bank(c, bank, t_ref, run, grid, n_t);
    if (st != FT_OK) return st;
    run.sum_mode = opts->sum_mode;
    run.precision = opts->precision;
    hipError_t e;

    // tile choice and LDS window for the grid kernel
    int tile = -1;
    if (grid) {
        const int64_t n0 = bank->n_f0, n1 = bank->n_f1, ns = bank->n_sky;
        if (opts->tile != 0) {
            if (opts->tile < 1 || opts->tile > tile_count()) return fail(c, FT_E_INVALID, "unknown tile %d", opts->tile);
            tile = opts->tile - 1;
        } else {
            tile = choose_tile(n0, n1, run.eta < 1e-4);
        }
        TileCfg cfg = tile_cfg(tile);
        if (cfg.L > 1 && !(run.eta < 1e-4)) {
            tile = 1;
            cfg = tile_cfg(tile);
        }
        const double T = c->t_sft;
        double dt_absmax = 0.0;
        for (double t : c->t_mid_h) dt_absmax = std::max(dt_absmax, std::fabs(t - t_ref));
        double span_f0 = 0.0;
        for (int64_t i0 = 0; i0 < n0; i0 += 64 * cfg.L) {
            const int64_t i1 = std::min<int64_t>(i0 + 64 * cfg.L, n0) - 1;
            span_f0 = std::max(span_f0, c->f0_h[i1] - c->f0_h[i0]);
        }
        double span_f1 = 0.0;
        for (int64_t j0 = 0; j0 < n1; j0 += cfg.JT) {
            double lo = c->f1_h[j0], hi = lo;
            for (int64_t j = j0; j < std::min<int64_t>(j0 + cfg.JT, n1); ++j) {
                lo = std::min(lo, c->f1_h[j]);
                hi = std::max(hi, c->f1_h[j]);
            }
            span_f1 = std::max(span_f1, hi - lo);
        }
        double diam = 0.0;
        const std::vector<double> &st = c->sky_tile_h;
        for (int64_t s0 = 0; s0 < ns; s0 += cfg.NW)
            for (int64_t a = s0; a < std::min<int64_t>(s0 + cfg.NW, ns); ++a)
                for (int64_t b2 = a + 1; b2 < std::min<int64_t>(s0 + cfg.NW, ns); ++b2) {
                    const double dx = st[3 * a] - st[3 * b2];
                    const double dy = st[3 * a + 1] - st[3 * b2 + 1];
                    const double dz = st[3 * a + 2] - st[3 * b2 + 2];
                    diam = std::max(diam, std::sqrt(dx * dx + dy * dy + dz * dz));
                }
        double f1_absmax = 0.0;
        for (double f : c->f1_h) f1_absmax = std::max(f1_absmax, std::fabs(f));
        const double a_max = c->f0_h[n0 - 1] + f1_absmax * dt_absmax;
        const double width = (span_f0 + span_f1 * dt_absmax) * (1.0 + c->vmax) * T +
                             a_max * c->vmax * diam * (1.0 + 1e-9) * T;
        const double wt = std::ceil(width * (1.0 + 1e-9)) + 3.0 + cfg.L;
        const double wtp = std::ceil(wt / 64.0) * 64.0;
        // A window beyond the LDS budget (extreme Doppler spread or a very
        // wide f1 tile) falls back to the direct kernel.
        if (2.0 * wtp * cfg.KS * 4.0 + (double)tile_static_lds(tile) > 150.0 * 1024.0) tile = -1;
        run.wt = (int32_t)std::min(wt, 1e9);
        run.wtp = (int32_t)std::min(wtp, 1e9);
        run.tiles_f0 = (int32_t)((n0 + 64 * cfg.L - 1) / (64 * cfg.L));
        run.tiles_f1 = (int32_t)((n1 + cfg.JT - 1) / cfg.JT);
        run.tiles_sky = (int32_t)((ns + cfg.NW - 1) / cfg.NW);
        if ((int64_t)run.tiles_f0 * run.tiles_f1 * run.tiles_sky >= 0x7fffffffLL)
            return fail(c, FT_E_UNSUPPORTED, "too many tiles");
    }

    // launch: clear flags, evaluate, select, re-sum, rank
    const int n_seg = opts->n_sub;
    const int k = opts->k;
    const int64_t cap = std::max<int64_t>(65536, (int64_t)64 * k * n_seg);
    st = ensure_select(c, n_seg, k, grid ? bank->n_f0 : n_t, cap);
    if (st != FT_OK) return st;
    if ((e = ensure(&c->d_edges, &c->cap_edges, edges.size())) != hipSuccess) return hip_fail(c, e, "alloc edges");
    e = hipMemcpyAsync(c->d_edges, edges.data(), edges.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_fill_u32(c->d_err, 0u, 1, c->stream);
    if (e == hipSuccess) e = launch_subband_map(c->d_f0, grid ? bank->n_f0 : n_t, c->d_edges, n_seg, c->d_seg, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev[0], c->stream);
    if (e == hipSuccess)
        e = !grid ? launch_eval_list(run, c->stream)
                  : tile < 0 ? launch_eval_grid_direct(run, c->stream) : launch_eval_grid(run, tile_cfg(tile), c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev[1], c->stream);
    const double N = (double)c->n_sft;
    const double rel_err = opts->sum_mode == FT_SUM_BLOCKED ? 40.0 * std::ldexp(1.0, -24) + 4.0 * N * std::ldexp(1.0, -53)
                                                            : (N + 8.0) * std::ldexp(1.0, -24) + 4.0 * N * std::ldexp(1.0, -53);
    SelectBufs sb = select_bufs(c, cap);
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
    return FT_OK;
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
        const int64_t cap = (int64_t)total + 1024;
        st = ensure_select(c, c->last_nsub, c->last_k, c->last_grid ? c->last_run.n_f0 : c->last_run.n_list, cap);
        if (st != FT_OK) return st;
        c->last_run.err = c->d_err;
        c->last_cap = cap;
        SelectBufs sb = select_bufs(c, cap);
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

ft_status ft_bins(ft_ctx c, const ft_bank *bank, double t_ref, int32_t precision, int32_t *bins)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    if (!bins) return fail(c, FT_E_INVALID, "bins is null");
    if (precision < FT_INDEX_FP64 || precision > FT_INDEX_GUARDED) return fail(c, FT_E_INVALID, "unknown precision");
    if (bank && bank->kind != FT_BANK_LIST) return fail(c, FT_E_UNSUPPORTED, "ft_bins takes a LIST bank");
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
                                    int64_t *n_mismatch)
{
    if (!c) return FT_E_INVALID;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FT_E_DEVICE, "hipSetDevice");
    if (!n_mismatch) return fail(c, FT_E_INVALID, "n_mismatch is null");
    if (precision < FT_INDEX_FP64 || precision > FT_INDEX_GUARDED) return fail(c, FT_E_INVALID, "unknown precision");
    EvalRun run;
    bool grid;
    int64_t n_t;
    ft_status st = prepare_bank(c, bank, t_ref, run, grid, n_t);
    if (st != FT_OK) return st;
    unsigned long long cnt = 0;
    hipError_t e = hipMemsetAsync(c->d_count, 0, sizeof cnt, c->stream);
    if (e == hipSuccess) e = launch_count_mismatch(run, grid, precision, c->d_count, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&cnt, c->d_count, sizeof cnt, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "count mismatches");
    *n_mismatch = (int64_t)cnt;
    c->have_eval = false;
    return FT_OK;
}

}  // extern "C"
