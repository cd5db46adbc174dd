// C-ABI of libtopk: context, parameters, workspace layout, argument checks and
// the launch plan of the single-instance selection.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <ctype.h>
#include <errno.h>
#include <stdio.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/topk.h"
#include "select.hpp"
#include "sort.hpp"
#include "ctx.hpp"

using namespace topk;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x, size_t a = ALIGN) { return (x + a - 1) / a * a; }

struct Layout {
    size_t state, hs, seg, band[4], trace, sort, total;
    uint32_t band_cap, band_alloc;
};

Layout make_layout(const topk_ctx *c, uint64_t n, uint32_t flags)
{
    Layout L{};
    size_t off = 0;
    L.state = off;
    off = align_up(off + sizeof(State));
    L.hs = off;
    off = align_up(off + (size_t)S_MAX * sizeof(uint64_t));
    L.seg = off;
    off = align_up(off + (size_t)NSEG * sizeof(uint32_t));
    uint64_t cap = n / (uint64_t)c->band_div + 65536;
    if (cap > n) cap = n;
    if (n <= (uint64_t)c->t_fin) cap = 0;
    L.band_cap = (uint32_t)cap;
    L.band_alloc = (uint32_t)((cap + 63) / 64 * 64);
    for (int i = 0; i < 4; ++i) {
        L.band[i] = off;
        off = align_up(off + (size_t)L.band_alloc * sizeof(uint32_t));
    }
    L.trace = off;
    if (flags & TOPK_TRACE) off = align_up(off + (size_t)R_TRACE * TRACE_STRIDE * sizeof(uint32_t));
    L.sort = off;
    if (flags & TOPK_SORTED) off = align_up(off + sort_ws_bytes(n));
    L.total = off;
    return L;
}

// Pivot ranks, as in the device code; used only for the host's round estimate.
void est_ranks(uint64_t s, uint64_t k, uint64_t n, uint64_t c_num, int64_t &lo, int64_t &hi)
{
    const uint64_t m_lo = k * s / n, m_hi = (k * s + n - 1) / n;
    const double d = ceil((double)c_num / 4.0 * sqrt((double)m_hi * (double)(s - m_lo) / (double)s));
    lo = (int64_t)m_lo - (int64_t)d - 1;
    hi = (int64_t)m_hi + (int64_t)d + 1;
}

// Expected subproblem sizes of the multi-workgroup rounds: the band of a
// round holds about (hi - lo) / s of the round's input.
int plan_rounds(const topk_ctx *c, uint64_t n, uint64_t k, double *sizes, int max_r)
{
    int r = 0;
    double nr = (double)n, kr = (double)k;
    while (r < max_r && nr > (double)c->t_fin) {
        sizes[r++] = nr;
        const double s = nr < (double)c->s_target ? nr : (double)c->s_target;
        int64_t lo, hi;
        uint64_t ki = (uint64_t)(kr < 1 ? 1 : kr), ni = (uint64_t)nr;
        if (ki > ni) ki = ni;
        est_ranks((uint64_t)s, ki, ni, (uint64_t)c->c_num, lo, hi);
        const double flo = lo > 0 ? (double)lo / s : 0.0;
        const double fhi = hi + 1 < (int64_t)s ? (double)(hi + 1) / s : 1.0;
        const double nb = (fhi - flo) * nr;
        kr -= flo * nr;
        nr = nb;
        if (nr <= (double)c->tail_max) break;
    }
    return r;
}

void set_defaults(topk_ctx *c)
{
    c->s_target = 4096;
    c->c_num = 16;
    c->t_fin = 16384;
    c->r_max = 24;
    c->r_fast = -1;
    c->band_div = 4;
    c->tail_max = 65536;
    c->timing = 0;
    c->bt_s_target = 1024;
    c->bt_c_num = 12;
    c->bt_wg_per_cu = 4;
    c->bt_attempts = 4;
    c->bt_fast = 1;
    c->bt_tile = 16;
    c->fq_mode = 0;
    for (int i = 0; i < TOPK_BT_NCLS; ++i) c->bt_s_cls[i] = c->bt_c_cls[i] = c->bt_t_cls[i] = -1;
}

// The tuning parameters (what topk_save_tuning writes), in a fixed order.
struct ParamRef { const char *name; int64_t topk_ctx::*field; };
const ParamRef TUNING[] = {
    {"s_target", &topk_ctx::s_target}, {"c_num", &topk_ctx::c_num}, {"t_fin", &topk_ctx::t_fin},
    {"r_max", &topk_ctx::r_max}, {"r_fast", &topk_ctx::r_fast}, {"band_div", &topk_ctx::band_div},
    {"tail_max", &topk_ctx::tail_max}, {"bt_s_target", &topk_ctx::bt_s_target},
    {"bt_c_num", &topk_ctx::bt_c_num}, {"bt_wg_per_cu", &topk_ctx::bt_wg_per_cu},
    {"bt_attempts", &topk_ctx::bt_attempts}, {"bt_fast", &topk_ctx::bt_fast},
    {"bt_tile", &topk_ctx::bt_tile}, {"fq_mode", &topk_ctx::fq_mode},
};

// "bt_s_target@C" / "bt_c_num@C" / "bt_tile@C": the override of row-length class C.
int64_t *cls_param(topk_ctx *c, const char *name)
{
    const char *at = strchr(name, '@');
    if (!at) return nullptr;
    const size_t len = (size_t)(at - name);
    int64_t *arr = nullptr;
    if (len == 11 && strncmp(name, "bt_s_target", 11) == 0) arr = c->bt_s_cls;
    else if (len == 8 && strncmp(name, "bt_c_num", 8) == 0) arr = c->bt_c_cls;
    else if (len == 7 && strncmp(name, "bt_tile", 7) == 0) arr = c->bt_t_cls;
    if (!arr || !at[1]) return nullptr;
    char *end = nullptr;
    const long cls = strtol(at + 1, &end, 10);
    if (*end || cls < 0 || cls >= TOPK_BT_NCLS) return nullptr;
    return arr + cls;
}

int check_device(int device, int *num_cu)
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return TOPK_E_HIP;
    if (strncmp(p.gcnArchName, "gfx950", 6) != 0) return TOPK_E_UNSUPPORTED;
    *num_cu = p.multiProcessorCount;
    return TOPK_OK;
}

template <typename K>
int select_common(topk_ctx *c, const K *keys, uint64_t n, uint64_t k, uint32_t flags,
                  uint32_t *out_idx, uint32_t *out_keys, uint32_t *kth_key,
                  uint32_t *kth_idx, uint32_t *status, void *ws, size_t ws_bytes,
                  hipStream_t stream, bool is_f32)
{
    if (!c || !keys || !out_idx || !kth_key || !kth_idx || !ws) return TOPK_E_INVALID;
    if (n == 0 || k == 0 || k > n || n > 0xFFFFFFFFull) return TOPK_E_INVALID;
    if (flags & ~(TOPK_LARGEST | TOPK_WRITE_KEYS | TOPK_TRACE | TOPK_SORTED)) return TOPK_E_INVALID;
    if ((flags & TOPK_WRITE_KEYS) && !out_keys) return TOPK_E_INVALID;
    if (((uintptr_t)keys & 3u) || ((uintptr_t)ws & (ALIGN - 1))) return TOPK_E_INVALID;
    const Layout L = make_layout(c, n, flags);
    if (ws_bytes < L.total) return TOPK_E_WORKSPACE;
    char *w = (char *)ws;
    SelArgs a{};
    a.keys = (const uint32_t *)keys;
    a.n = (uint32_t)n;
    a.k = (uint32_t)k;
    a.flags = flags;
    a.out_idx = out_idx;
    a.out_keys = (flags & TOPK_WRITE_KEYS) ? out_keys : nullptr;
    a.kth_key = kth_key;
    a.kth_idx = kth_idx;
    a.status = status;
    a.st = (State *)(w + L.state);
    a.hs_buf = (uint64_t *)(w + L.hs);
    a.seg_cnt = (uint32_t *)(w + L.seg);
    a.band_cap = L.band_cap;
    a.band_ord[0] = (uint32_t *)(w + L.band[0]);
    a.band_idx[0] = (uint32_t *)(w + L.band[1]);
    a.band_ord[1] = (uint32_t *)(w + L.band[2]);
    a.band_idx[1] = (uint32_t *)(w + L.band[3]);
    a.trace_pos = (flags & TOPK_TRACE) ? (uint32_t *)(w + L.trace) : nullptr;
    a.s_target = (uint32_t)c->s_target;
    a.c_num0 = (uint32_t)c->c_num;
    a.t_fin = (uint32_t)c->t_fin;
    a.r_max = (uint32_t)c->r_max;
    a.seed = c->seed;

    SelLaunch P{};
    P.is_f32 = is_f32;
    P.largest = (flags & TOPK_LARGEST) != 0;
    double sizes[8];
    int r = plan_rounds(c, n, k, sizes, 8);
    if (c->r_fast >= 0) r = (int)c->r_fast;
    P.r_fast = r;
    const int gmax = sweep_max_grid(is_f32, (flags & TOPK_LARGEST) != 0, c->num_cu);
    for (int i = 0; i < 8; ++i) {
        // every sweep gets the full resident grid: a round repeated on a
        // larger subproblem than planned (a miss re-sweeps its whole input)
        // keeps every CU, and workgroups without a wave-tile exit at once.
        // Only the first round's grid is bounded by its wave-tiles.
        const uint64_t t = (uint64_t)((n + SW_TILE_IN - 1) / SW_TILE_IN) + 1;
        P.sweep_grid[i] = (i == 0 && t < (uint64_t)gmax) ? (int)t : gmax;
    }
    if (hipSetDevice(c->device) != hipSuccess) return TOPK_E_HIP;
    KernelTimer tm{};
    if (c->timing > 0) {
        const int need = c->ev_used + 2 * P.r_fast + 4;
        while ((int)c->ev_kind.size() < need) {
            hipEvent_t e0, e1;
            if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
                return TOPK_E_HIP;
            c->ev.push_back(e0);
            c->ev.push_back(e1);
            c->ev_kind.push_back(-1);
        }
        tm.level = (int)c->timing;
        tm.ev = c->ev.data();
        tm.kind = c->ev_kind.data();
        tm.cap = (int)c->ev_kind.size();
        tm.used = c->ev_used;
    }
    hipError_t e = launch_select(a, P, stream, c->timing > 0 ? &tm : nullptr);
    if (c->timing > 0) c->ev_used = tm.used;
    if (e == hipSuccess && (flags & TOPK_SORTED))
        e = sort_selected((const uint32_t *)keys, n, is_f32, (flags & TOPK_LARGEST) != 0, out_idx,
                          a.out_keys, k, w + L.sort, stream);
    return e == hipSuccess ? TOPK_OK : TOPK_E_HIP;
}

}  // namespace

extern "C" {

int topk_create(topk_ctx **out, int hip_device, uint64_t seed)
{
    if (!out) return TOPK_E_INVALID;
    *out = nullptr;
    int ncu = 0;
    int rc = check_device(hip_device, &ncu);
    if (rc != TOPK_OK) return rc;
    rc = topk_bt_scratch_setup(hip_device);
    if (rc != TOPK_OK) return rc;
    topk_ctx *c = new (std::nothrow) topk_ctx;
    if (!c) return TOPK_E_INVALID;
    c->device = hip_device;
    c->seed = seed;
    set_defaults(c);
    c->num_cu = ncu;
    *out = c;
    return TOPK_OK;
}

void topk_destroy(topk_ctx *c)
{
    if (!c) return;
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    delete c;
}

int topk_set_param(topk_ctx *c, const char *name, int64_t v)
{
    if (!c || !name) return TOPK_E_INVALID;
    struct { const char *n; int64_t *p; int64_t lo, hi; } tab[] = {
        {"s_target", &c->s_target, 16, 8192},
        {"c_num", &c->c_num, 0, 4096},
        {"t_fin", &c->t_fin, 1, T_FIN_MAX},
        {"r_max", &c->r_max, 1, 32},
        {"r_fast", &c->r_fast, -1, 8},
        {"band_div", &c->band_div, 1, 64},
        {"tail_max", &c->tail_max, 0, (int64_t)1 << 32},
        {"timing", &c->timing, 0, 2},
        {"bt_s_target", &c->bt_s_target, 64, 2048},
        {"bt_c_num", &c->bt_c_num, 4, 4096},
        {"bt_wg_per_cu", &c->bt_wg_per_cu, 1, 8},
        {"bt_attempts", &c->bt_attempts, 1, 16},
        {"bt_fast", &c->bt_fast, 0, 1},
        {"bt_tile", &c->bt_tile, 8, 16},
        {"fq_mode", &c->fq_mode, 0, 3},
    };
    if (strcmp(name, "seed") == 0) { c->seed = (uint64_t)v; return TOPK_OK; }
    int64_t *cls = cls_param(c, name);
    if (cls) {
        // -1 removes the override; otherwise the range of the global parameter
        int64_t lo = 4, hi = 4096;
        if (name[3] == 's') lo = 64, hi = 2048;
        else if (name[3] == 't') lo = 8, hi = 16;
        if (v != -1 && (v < lo || v > hi || (name[3] == 't' && v != 8 && v != 16)))
            return TOPK_E_INVALID;
        *cls = v;
        return TOPK_OK;
    }
    for (auto &e : tab) {
        if (strcmp(name, e.n) == 0) {
            if (v < e.lo || v > e.hi) return TOPK_E_INVALID;
            if (e.p == &c->bt_tile && v != 8 && v != 16) return TOPK_E_INVALID;
            *e.p = v;
            return TOPK_OK;
        }
    }
    return TOPK_E_INVALID;
}

int topk_get_param(const topk_ctx *c, const char *name, int64_t *v)
{
    if (!c || !name || !v) return TOPK_E_INVALID;
    if (strcmp(name, "seed") == 0) { *v = (int64_t)c->seed; return TOPK_OK; }
    if (const int64_t *cls = cls_param(const_cast<topk_ctx *>(c), name)) { *v = *cls; return TOPK_OK; }
    const struct { const char *n; int64_t val; } tab[] = {
        {"s_target", c->s_target}, {"c_num", c->c_num}, {"t_fin", c->t_fin},
        {"r_max", c->r_max}, {"r_fast", c->r_fast}, {"band_div", c->band_div},
        {"tail_max", c->tail_max}, {"timing", c->timing},
        {"bt_s_target", c->bt_s_target}, {"bt_c_num", c->bt_c_num},
        {"bt_wg_per_cu", c->bt_wg_per_cu}, {"bt_attempts", c->bt_attempts},
        {"bt_fast", c->bt_fast}, {"bt_tile", c->bt_tile}, {"fq_mode", c->fq_mode},
    };
    for (auto &e : tab) {
        if (strcmp(name, e.n) == 0) { *v = e.val; return TOPK_OK; }
    }
    return TOPK_E_INVALID;
}

size_t topk_workspace_bytes(const topk_ctx *c, uint64_t n, uint32_t flags)
{
    if (!c) return 0;
    return make_layout(c, n, flags).total;
}

int topk_select_u32(topk_ctx *c, const uint32_t *keys, uint64_t n, uint64_t k,
                    uint32_t flags, uint32_t *out_idx, uint32_t *out_keys,
                    uint32_t *kth_key, uint32_t *kth_idx, uint32_t *status,
                    void *ws, size_t ws_bytes, hipStream_t stream)
{
    return select_common(c, keys, n, k, flags, out_idx, out_keys, kth_key, kth_idx,
                         status, ws, ws_bytes, stream, false);
}

int topk_select_f32(topk_ctx *c, const float *keys, uint64_t n, uint64_t k,
                    uint32_t flags, uint32_t *out_idx, float *out_keys,
                    float *kth_key, uint32_t *kth_idx, uint32_t *status,
                    void *ws, size_t ws_bytes, hipStream_t stream)
{
    return select_common(c, keys, n, k, flags, out_idx, (uint32_t *)out_keys,
                         (uint32_t *)kth_key, kth_idx, status, ws, ws_bytes, stream, true);
}

int topk_trace_rounds(const topk_ctx *c, const void *ws, uint64_t n,
                      topk_round_record *out, uint32_t max, uint32_t *count,
                      hipStream_t stream)
{
    (void)n;
    if (!c || !ws || !out || !count) return TOPK_E_INVALID;
    static_assert(sizeof(RoundRec) == sizeof(topk_round_record), "record layout");
    State st;
    if (hipMemcpyAsync(&st, ws, sizeof(State), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return TOPK_E_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return TOPK_E_HIP;
    uint32_t m = st.nrec < (uint32_t)R_TRACE ? st.nrec : (uint32_t)R_TRACE;
    if (m > max) m = max;
    memcpy(out, st.rec, m * sizeof(RoundRec));
    *count = st.nrec;
    return TOPK_OK;
}

int topk_trace_sample(const topk_ctx *c, const void *ws, uint64_t n, uint32_t tag,
                      uint32_t *out_pos, uint32_t cap, uint32_t *count, hipStream_t stream)
{
    if (!c || !ws || !out_pos || !count || tag >= (uint32_t)R_TRACE) return TOPK_E_INVALID;
    const Layout L = make_layout(c, n, TOPK_TRACE);
    State st;
    if (hipMemcpyAsync(&st, ws, sizeof(State), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return TOPK_E_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return TOPK_E_HIP;
    if (tag >= st.nrec) { *count = 0; return TOPK_OK; }
    uint32_t s = st.rec[tag].s;
    *count = s;
    if (s > cap) s = cap;
    const char *src = (const char *)ws + L.trace + (size_t)tag * TRACE_STRIDE * sizeof(uint32_t);
    if (hipMemcpyAsync(out_pos, src, (size_t)s * sizeof(uint32_t), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return TOPK_E_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return TOPK_E_HIP;
    return TOPK_OK;
}

int topk_kernel_times(topk_ctx *c, float *ms, int32_t *kind, uint32_t max, uint32_t *count)
{
    if (!c || !count || (max && (!ms || !kind))) return TOPK_E_INVALID;
    const uint32_t m = (uint32_t)c->ev_used;
    for (uint32_t i = 0; i < m && i < max; ++i) {
        if (hipEventSynchronize(c->ev[2 * i + 1]) != hipSuccess) return TOPK_E_HIP;
        float t = 0.f;
        if (hipEventElapsedTime(&t, c->ev[2 * i], c->ev[2 * i + 1]) != hipSuccess) return TOPK_E_HIP;
        ms[i] = t;
        kind[i] = c->ev_kind[i];
    }
    *count = m;
    c->ev_used = 0;
    return TOPK_OK;
}

int topk_tune_f32(topk_ctx *c, const float *keys, uint64_t n, uint64_t k, uint32_t flags,
                  uint32_t *out_idx, float *kth_key, uint32_t *kth_idx, void *ws,
                  size_t ws_bytes, uint32_t reps, hipStream_t stream)
{
    if (!c || reps == 0 || reps > 100) return TOPK_E_INVALID;
    if (flags & ~(uint32_t)TOPK_LARGEST) return TOPK_E_INVALID;
    // the workspace size does not depend on s_target or c_num
    auto call = [&]() {
        return select_common(c, (const uint32_t *)keys, n, k, flags, out_idx, nullptr,
                             (uint32_t *)kth_key, kth_idx, nullptr, ws, ws_bytes, stream, true);
    };
    int rc = call();                    // argument checks, and a warm-up
    if (rc != TOPK_OK) return rc;
    if (hipSetDevice(c->device) != hipSuccess) return TOPK_E_HIP;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return TOPK_E_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return TOPK_E_HIP; }
    const int64_t keep_s = c->s_target, keep_c = c->c_num;
    const int64_t s_cand[] = {2048, 4096, 8192};
    const int64_t c_cand[] = {8, 12, 16, 24};
    float best = -1.0f;
    int64_t bs = keep_s, bc = keep_c;
    for (int64_t sv : s_cand) {
        for (int64_t cv : c_cand) {
            c->s_target = sv;
            c->c_num = cv;
            std::vector<float> t;
            for (uint32_t i = 0; i < reps && rc == TOPK_OK; ++i) {
                float ms = 0.0f;
                if (hipEventRecord(e0, stream) != hipSuccess) rc = TOPK_E_HIP;
                if (rc == TOPK_OK) rc = call();
                if (rc == TOPK_OK && (hipEventRecord(e1, stream) != hipSuccess ||
                                      hipEventSynchronize(e1) != hipSuccess ||
                                      hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = TOPK_E_HIP;
                t.push_back(ms);
            }
            if (rc != TOPK_OK) break;
            // the mean, so that a pair whose rounds sometimes miss (and
            // repeat) pays for it
            float mean = 0.0f;
            for (float x : t) mean += x;
            mean /= (float)t.size();
            if (best < 0.0f || mean < best) { best = mean; bs = sv; bc = cv; }
        }
        if (rc != TOPK_OK) break;
    }
    c->s_target = rc == TOPK_OK ? bs : keep_s;
    c->c_num = rc == TOPK_OK ? bc : keep_c;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int topk_save_tuning(const topk_ctx *c, const char *path)
{
    if (!c || !path) return TOPK_E_INVALID;
    FILE *f = fopen(path, "w");
    if (!f) return TOPK_E_INVALID;
    bool first = true;
    auto put = [&](const char *name, int64_t v) {
        fprintf(f, "%s\n  \"%s\": %lld", first ? "{" : ",", name, (long long)v);
        first = false;
    };
    for (const ParamRef &p : TUNING) put(p.name, c->*p.field);
    char name[32];
    for (int i = 0; i < TOPK_BT_NCLS; ++i) {
        if (c->bt_s_cls[i] >= 0) { snprintf(name, sizeof name, "bt_s_target@%d", i); put(name, c->bt_s_cls[i]); }
        if (c->bt_c_cls[i] >= 0) { snprintf(name, sizeof name, "bt_c_num@%d", i); put(name, c->bt_c_cls[i]); }
        if (c->bt_t_cls[i] >= 0) { snprintf(name, sizeof name, "bt_tile@%d", i); put(name, c->bt_t_cls[i]); }
    }
    fprintf(f, "%s\n}\n", first ? "{" : "");
    const bool ok = fclose(f) == 0;
    return ok ? TOPK_OK : TOPK_E_INVALID;
}

int topk_load_tuning(topk_ctx *c, const char *path)
{
    if (!c) return TOPK_E_INVALID;
    if (!path) {
        const int64_t tm = c->timing;
        set_defaults(c);
        c->timing = tm;
        return TOPK_OK;
    }
    FILE *f = fopen(path, "r");
    if (!f) return TOPK_E_INVALID;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    // a flat JSON object of "name": integer pairs
    std::vector<std::pair<std::string, int64_t>> kv;
    size_t i = 0;
    auto ws = [&]() { while (i < text.size() && isspace((unsigned char)text[i])) ++i; };
    ws();
    if (i >= text.size() || text[i] != '{') return TOPK_E_INVALID;
    ++i;
    ws();
    if (i < text.size() && text[i] == '}') {
        ++i;
    } else {
        for (;;) {
            ws();
            if (i >= text.size() || text[i] != '"') return TOPK_E_INVALID;
            const size_t e = text.find('"', i + 1);
            if (e == std::string::npos) return TOPK_E_INVALID;
            std::string name = text.substr(i + 1, e - i - 1);
            i = e + 1;
            ws();
            if (i >= text.size() || text[i] != ':') return TOPK_E_INVALID;
            ++i;
            ws();
            char *end = nullptr;
            errno = 0;
            const long long v = strtoll(text.c_str() + i, &end, 10);
            if (end == text.c_str() + i || errno) return TOPK_E_INVALID;
            i = (size_t)(end - text.c_str());
            kv.emplace_back(name, (int64_t)v);
            ws();
            if (i < text.size() && text[i] == ',') { ++i; continue; }
            if (i < text.size() && text[i] == '}') { ++i; break; }
            return TOPK_E_INVALID;
        }
    }
    ws();
    if (i != text.size()) return TOPK_E_INVALID;
    // all or nothing: apply to a copy of the parameters, then keep them
    topk_ctx *t = new (std::nothrow) topk_ctx;
    if (!t) return TOPK_E_INVALID;
    for (const ParamRef &p : TUNING) t->*p.field = c->*p.field;
    memcpy(t->bt_s_cls, c->bt_s_cls, sizeof t->bt_s_cls);
    memcpy(t->bt_c_cls, c->bt_c_cls, sizeof t->bt_c_cls);
    memcpy(t->bt_t_cls, c->bt_t_cls, sizeof t->bt_t_cls);
    t->seed = c->seed;
    t->timing = c->timing;
    int rc = TOPK_OK;
    for (auto &p : kv) {
        if (p.first == "seed" || p.first == "timing" || topk_set_param(t, p.first.c_str(), p.second) != TOPK_OK) {
            rc = TOPK_E_INVALID;
            break;
        }
    }
    if (rc == TOPK_OK) {
        for (const ParamRef &p : TUNING) c->*p.field = t->*p.field;
        memcpy(c->bt_s_cls, t->bt_s_cls, sizeof c->bt_s_cls);
        memcpy(c->bt_c_cls, t->bt_c_cls, sizeof c->bt_c_cls);
        memcpy(c->bt_t_cls, t->bt_t_cls, sizeof c->bt_t_cls);
    }
    delete t;
    return rc;
}

const char *topk_strerror(int code)
{
    switch (code) {
    case TOPK_OK: return "ok";
    case TOPK_E_INVALID: return "invalid argument";
    case TOPK_E_WORKSPACE: return "workspace too small";
    case TOPK_E_HIP: return "HIP runtime error";
    case TOPK_E_UNSUPPORTED: return "device is not gfx950";
    default: return "unknown error";
    }
}

}  // extern "C"
