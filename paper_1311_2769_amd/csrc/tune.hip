// Launch-shape autotuner and its cache.
//
// The vote kernels take a launch shape (phi0 rows per LDS tile, workgroup
// size, and for a single event the number of hit chunks per tile); results
// never depend on it, speed does.  hough_autotune times every supported shape
// on the caller's resident hits, keeps the fastest and appends it to a cache
// file, one JSON object per line:
//
//   {"device": "gfx950/256", "grid": [1, 1024, 512], "acc": "i32", "which": 1,
//    "hits_log2": 23, "rows": 32, "threads": 512, "split": 1, "ms": 2.006}
//
// keyed by device (architecture and compute-unit count), grid dimensions,
// accumulator type, launch kind (0 single event, 1 batch) and the hit count
// rounded up to a power of two.  hough_ctx_create applies the entry of its
// key whose hit bucket is nearest to its max_hits (the last such line wins).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hough.h"
#include "hough_impl.h"

namespace hough {
namespace {

const char *skip_ws(const char *p) {
    while (*p == ' ' || *p == '\t')
        ++p;
    return p;
}

// Position just after `"name":` in a flat JSON object, or nullptr.
const char *field(const char *line, const char *name) {
    const size_t n = std::strlen(name);
    for (const char *p = std::strchr(line, '"'); p; p = std::strchr(p + 1, '"')) {
        if (std::strncmp(p + 1, name, n) == 0 && p[n + 1] == '"') {
            const char *q = skip_ws(p + n + 2);
            if (*q == ':')
                return skip_ws(q + 1);
        }
    }
    return nullptr;
}

bool read_string(const char *p, std::string *out) {
    if (!p || *p != '"')
        return false;
    const char *e = std::strchr(p + 1, '"');
    if (!e)
        return false;
    out->assign(p + 1, e);
    return true;
}

bool read_long(const char *p, long long *out) {
    if (!p)
        return false;
    char *end = nullptr;
    const long long v = std::strtoll(p, &end, 10);
    if (end == p)
        return false;
    *out = v;
    return true;
}

bool read_int(const char *line, const char *name, int *out) {
    long long v = 0;
    if (!read_long(field(line, name), &v) || v < INT32_MIN || v > INT32_MAX)
        return false;
    *out = static_cast<int>(v);
    return true;
}

bool read_dims(const char *p, int dims[3]) {
    if (!p || *p != '[')
        return false;
    ++p;
    for (int i = 0; i < 3; ++i) {
        p = skip_ws(p);
        char *end = nullptr;
        const long v = std::strtol(p, &end, 10);
        if (end == p)
            return false;
        dims[i] = static_cast<int>(v);
        p = skip_ws(end);
        if (i < 2) {
            if (*p != ',')
                return false;
            ++p;
        }
    }
    return *p == ']';
}

}  // namespace

int tune_hits_log2(int64_t hits) {
    int b = 0;
    while (b < 62 && (int64_t{1} << b) < hits)
        ++b;
    return b;
}

bool tune_parse(const char *line, TuneEntry *e) {
    int dims[3];
    std::string acc;
    if (!read_string(field(line, "device"), &e->device) || !read_dims(field(line, "grid"), dims) ||
        !read_string(field(line, "acc"), &acc))
        return false;
    e->n_d0 = dims[0];
    e->n_phi = dims[1];
    e->n_kappa = dims[2];
    if (acc == "i32")
        e->acc = HOUGH_ACC_I32;
    else if (acc == "u16")
        e->acc = HOUGH_ACC_U16;
    else
        return false;
    if (!read_int(line, "which", &e->which) || !read_int(line, "hits_log2", &e->hits_log2) ||
        !read_int(line, "rows", &e->rows) || !read_int(line, "threads", &e->threads) ||
        !read_int(line, "split", &e->split))
        return false;
    const char *ms = field(line, "ms");
    e->ms = ms ? std::strtod(ms, nullptr) : 0.0;
    return true;
}

std::string tune_format(const TuneEntry &e) {
    char buf[512];
    std::snprintf(buf, sizeof buf,
                  "{\"device\": \"%s\", \"grid\": [%d, %d, %d], \"acc\": \"%s\", \"which\": %d, "
                  "\"hits_log2\": %d, \"rows\": %d, \"threads\": %d, \"split\": %d, \"ms\": %.4f}\n",
                  e.device.c_str(), e.n_d0, e.n_phi, e.n_kappa, e.acc == HOUGH_ACC_U16 ? "u16" : "i32", e.which,
                  e.hits_log2, e.rows, e.threads, e.split, e.ms);
    return buf;
}

bool tune_lookup(const char *path, const TuneEntry &key, TuneEntry *out) {
    if (!path || !*path)
        return false;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return false;
    bool found = false;
    int best_dist = 0;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        TuneEntry e;
        if (!tune_parse(line, &e))
            continue;
        if (e.device != key.device || e.n_d0 != key.n_d0 || e.n_phi != key.n_phi || e.n_kappa != key.n_kappa ||
            e.acc != key.acc || e.which != key.which)
            continue;
        const int dist = std::abs(e.hits_log2 - key.hits_log2);
        if (!found || dist <= best_dist) {
            *out = e;
            best_dist = dist;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

bool tune_append(const char *path, const TuneEntry &e) {
    if (!path || !*path)
        return false;
    FILE *f = std::fopen(path, "a");
    if (!f)
        return false;
    const std::string s = tune_format(e);
    const bool ok = std::fwrite(s.data(), 1, s.size(), f) == s.size();
    return std::fclose(f) == 0 && ok;
}

std::string device_tag(int device) {
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return "unknown";
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos)
        arch.resize(colon);
    return arch + "/" + std::to_string(prop.multiProcessorCount);
}

const char *tune_cache_path(const char *opt) {
    if (opt && *opt)
        return opt;
    const char *env = std::getenv("HOUGH_TUNE_CACHE");
    return (env && *env) ? env : nullptr;
}

}  // namespace hough

using namespace hough;

namespace {

float median(std::vector<float> v) {
    std::sort(v.begin(), v.end());
    return v.empty() ? 0.0f : v[v.size() / 2];
}

}  // namespace

extern "C" {

hough_status hough_tune_lookup(const char *cache_path, const char *device, const hough_grid *grid, int32_t which,
                               int64_t hits, int32_t *found, int32_t *rows, int32_t *threads, int32_t *split) {
    if (!device || !grid || !found || (which != 0 && which != 1) || hits < 0)
        return HOUGH_EINVAL;
    TuneEntry key;
    key.device = device;
    key.n_d0 = grid->n_d0;
    key.n_phi = grid->n_phi;
    key.n_kappa = grid->n_kappa;
    key.acc = grid->acc_type;
    key.which = which;
    key.hits_log2 = tune_hits_log2(hits);
    TuneEntry e;
    *found = tune_lookup(tune_cache_path(cache_path), key, &e) ? 1 : 0;
    if (*found) {
        if (rows)
            *rows = e.rows;
        if (threads)
            *threads = e.threads;
        if (split)
            *split = e.split;
    }
    return HOUGH_OK;
}

hough_status hough_autotune(hough_ctx *ctx, int32_t which, int32_t n_events, const int64_t *hit_off,
                            const float *x, const float *y, int32_t threshold, void *acc, hough_cand *cands,
                            const int64_t *cand_off, int32_t *n_found, int32_t reps, const char *cache_path,
                            void *stream, float *best_ms) {
    if (!ctx || (which != 0 && which != 1) || n_events < 1 || !hit_off || reps < 1 || reps > 1000)
        return HOUGH_EINVAL;
    if (which == 0 && !acc)
        return HOUGH_EINVAL;
    int32_t r0 = 0, t0 = 0, s0 = 0;
    hough_status st = hough_get_launch(ctx, which, &r0, &t0, &s0);
    if (st != HOUGH_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n_hits = which == 0 ? hit_off[1] - hit_off[0] : hit_off[n_events];
    if (which == 0 && (n_hits < 0 || n_hits > 0x7fffffffLL))
        return HOUGH_EINVAL;

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (which == 0) {
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0)
                (void)hipEventDestroy(e0);
            return HOUGH_EDEVICE;
        }
    }
    // One timed run of the current shape: the whole batch (timing mode), or
    // one single-event vote.
    auto run = [&](float *ms) -> hough_status {
        if (which == 1) {
            hough_status r = hough_event_batch(ctx, n_events, hit_off, x, y, threshold, acc, cands, cand_off,
                                               n_found, nullptr, stream);
            if (r != HOUGH_OK)
                return r;
            float v = 0.0f;
            return hough_get_timing(ctx, &v, ms);
        }
        const float *xe = x + hit_off[0];
        const float *ye = y + hit_off[0];
        if (hipEventRecord(e0, s) != hipSuccess)
            return HOUGH_EDEVICE;
        hough_status r = hough_vote(ctx, xe, ye, static_cast<int32_t>(n_hits), acc, nullptr, stream);
        if (r != HOUGH_OK)
            return r;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            return HOUGH_EDEVICE;
        return HOUGH_OK;
    };

    const int rows_c[] = {32, 64, 128};
    const int threads_c[] = {256, 512, 1024};
    const int split_c[] = {1, 2, 4, 8, 16};
    const int n_split = which == 0 ? 5 : 1;
    int br = r0, bt = t0, bs = s0;
    float best = INFINITY;
    if (which == 1)
        st = hough_set_timing(ctx, 1);
    for (int ri = 0; ri < 3 && st == HOUGH_OK; ++ri) {
        for (int ti = 0; ti < 3 && st == HOUGH_OK; ++ti) {
            for (int si = 0; si < n_split && st == HOUGH_OK; ++si) {
                if (hough_set_launch(ctx, which, rows_c[ri], threads_c[ti], split_c[si]) != HOUGH_OK)
                    continue;   // does not fit this grid or context
                std::vector<float> t;
                for (int k = 0; k <= reps && st == HOUGH_OK; ++k) {
                    float ms = 0.0f;
                    st = run(&ms);
                    if (k > 0)
                        t.push_back(ms);   // the first run warms up (and captures nothing in timing mode)
                }
                if (st != HOUGH_OK)
                    break;
                const float m = median(t);
                if (m < best) {
                    best = m;
                    br = rows_c[ri];
                    bt = threads_c[ti];
                    bs = split_c[si];
                }
            }
        }
    }
    if (which == 1)
        (void)hough_set_timing(ctx, 0);
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    const hough_status set = hough_set_launch(ctx, which, br, bt, bs);
    if (st != HOUGH_OK)
        return st;
    if (set != HOUGH_OK)
        return set;
    if (best_ms)
        *best_ms = best;
    const char *path = tune_cache_path(cache_path);
    if (path) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        TuneEntry e;
        e.device = device_tag(dev);
        hough_grid g{};
        ctx_grid(ctx, &g);
        e.n_d0 = g.n_d0;
        e.n_phi = g.n_phi;
        e.n_kappa = g.n_kappa;
        e.acc = g.acc_type;
        e.which = which;
        e.hits_log2 = tune_hits_log2(n_hits);
        e.rows = br;
        e.threads = bt;
        e.split = bs;
        e.ms = best;
        if (!tune_append(path, e))
            return HOUGH_EINVAL;   // the cache file cannot be written
    }
    return HOUGH_OK;
}

}  // extern "C"
