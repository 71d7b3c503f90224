// Schedule autotuner: for every valid (residues per lane, waves per
// workgroup) times the forward and the adjoint (or the fused step) separately
// with HIP events, and keeps the fastest of each as the plan's forward and
// adjoint schedules; choices can be kept in a small text cache.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "a2c_internal.h"

namespace a2c {
// retire_old: keep the replaced tables until the plan is destroyed (a graph
// captured before may use them); false frees them (the tuner's own candidates)
a2c_status plan_apply_forward_schedule(a2c_plan *p, int32_t K, int32_t W, hipStream_t s,
                                       bool retire_old);
a2c_status plan_apply_adjoint_schedule(a2c_plan *p, int32_t K, int32_t W, hipStream_t s,
                                       bool retire_old);
}

using namespace a2c;

namespace {

std::string cache_key(const a2c_plan *p, int from_coords)
{
    hipDeviceProp_t prop;
    std::string dev = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) dev = prop.gcnArchName;
    for (char &c : dev)
        if (c == ' ' || c == ':') c = '_';
    std::ostringstream k;
    k << dev << ' ' << (p->model == A2C_BACKBONE ? "backbone" : "fullatom") << ' ' << p->R << ' '
      << p->max_len << ' ' << p->n_chains << ' '
      << (from_coords == A2C_TUNE_MSE_STEP ? "mse" : from_coords ? "coords" : "recompute");
    return k.str();
}

// A cache line is "<key> K W [bK bW]": forward, then adjoint schedule (a line
// with two numbers gives both).  A line whose schedules a2c_plan_set_schedule
// would reject for this plan is skipped, as is anything after the numbers.
bool cache_lookup(const a2c_plan *p, const char *path, const std::string &key, int32_t &K,
                  int32_t &W, int32_t &bK, int32_t &bW)
{
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        if (line.compare(0, key.size(), key) != 0 || line.size() <= key.size() ||
            line[key.size()] != ' ')
            continue;
        int k = 0, w = 0, bk = 0, bw = 0, used = 0;
        const char *rest = line.c_str() + key.size();
        int n = std::sscanf(rest, " %d %d %d %d%n", &k, &w, &bk, &bw, &used);
        if (n != 4) {
            used = 0;
            n = std::sscanf(rest, " %d %d%n", &k, &w, &used) == 2 ? 2 : 0;
        }
        if (n == 2) bk = k, bw = w;
        const bool tail_blank = used > 0 && rest[std::strspn(rest + used, " \t\r") + used] == '\0';
        if (n != 0 && tail_blank && check_forward_schedule_args(p, k, w) == A2C_OK &&
            check_schedule_args(p, bk, bw) == A2C_OK) {
            K = k;
            W = w;
            bK = bk;
            bW = bw;
            found = true;  // the last valid matching line wins
        }
    }
    return found;
}

void cache_store(const char *path, const std::string &key, int32_t K, int32_t W, int32_t bK,
                 int32_t bW)
{
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    if (f) f << key << ' ' << K << ' ' << W << ' ' << bK << ' ' << bW << '\n';
}

// The forward, then the adjoint schedule (each setter leaves its schedule
// unchanged when it fails).
a2c_status apply_pair(a2c_plan *p, int32_t K, int32_t W, int32_t bK, int32_t bW, hipStream_t s,
                      bool retire_old)
{
    a2c_status st = plan_apply_forward_schedule(p, K, W, s, retire_old);
    if (st == A2C_OK) st = plan_apply_adjoint_schedule(p, bK, bW, s, retire_old);
    return st;
}

}  // namespace

extern "C" a2c_status a2c_plan_autotune(a2c_plan *p, const float *d_angles, float *d_coords,
                                        const float *d_grad_coords, float *d_grad_angles,
                                        int32_t from_coords, int32_t reps, const char *cache_path,
                                        int32_t *out_K, int32_t *out_W, void *stream)
{
    if (!p) {
        set_error("plan is NULL");
        return A2C_ERR_INVALID_ARG;
    }
    if (reps < 1) {
        set_error("reps must be >= 1");
        return A2C_ERR_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    if (p->R == 0) {
        if (out_K) *out_K = p->fs.K;
        if (out_W) *out_W = p->fs.W;
        return A2C_OK;
    }
    if (!d_angles || !d_coords || !d_grad_coords || !d_grad_angles) {
        set_error("NULL buffer");
        return A2C_ERR_INVALID_ARG;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device) {
        set_error("current device is not the plan's device");
        return A2C_ERR_STATE;
    }
    const std::string key = cache_key(p, from_coords);
    int32_t K = 0, W = 0, cK = 0, cW = 0;
    if (cache_lookup(p, cache_path, key, K, W, cK, cW)) {
        if (apply_pair(p, K, W, cK, cW, s, true) == A2C_OK) {
            if (out_K) *out_K = K;
            if (out_W) *out_W = W;
            return A2C_OK;
        }
    }
    const int Ks[4] = {1, 2, 4, 8};
    const int Ws[8] = {1, 2, 3, 4, 6, 8, 12, 16};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return hip_fail(hipGetLastError(), "hipEventCreate");
    // best of three timed trials (after one warm-up) of reps calls of part
    // 0 (forward) or 1 (adjoint / fused step)
    auto time_part = [&](int part, float &best) -> a2c_status {
        best = 1e30f;
        a2c_status rs = A2C_OK;
        for (int trial = 0; trial < 4 && rs == A2C_OK; ++trial) {
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps && rs == A2C_OK; ++r) {
                if (part == 0)
                    rs = a2c_forward(p, A2C_SCAN, d_angles, d_coords, nullptr, s);
                else if (from_coords == A2C_TUNE_MSE_STEP)  // d_grad_coords: the target
                    rs = a2c_mse_step(p, d_angles, d_grad_coords, d_coords, nullptr,
                                      d_grad_angles, s);
                else
                    rs = a2c_backward(p, A2C_SCAN, d_angles, from_coords ? d_coords : nullptr,
                                      d_grad_coords, d_grad_angles, nullptr, s);
            }
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess)
                return hip_fail(hipGetLastError(), "hipEventSynchronize");
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (trial > 0) best = std::min(best, ms);  // the first trial warms up
        }
        return rs;
    };
    float best_f = 1e30f, best_b = 1e30f;
    int32_t fK = p->fs.K, fW = p->fs.W, bK = p->bs.K, bW = p->bs.W;
    a2c_status st = A2C_OK;
    // The forward schedules, then the adjoint ones with the fastest forward in
    // place (its output feeds the coordinate-mode adjoint).  The first
    // candidate of each replaces the caller's schedule (retired: a graph may
    // hold it); later ones replace the tuner's own (freed).
    bool own_f = false, own_b = false;
    for (int part = 0; part < 2 && st == A2C_OK; ++part) {
        for (int k : Ks) {
            for (int w : Ws) {
                st = part == 0 ? check_forward_schedule_args(p, k, w)
                               : check_schedule_args(p, k, w);
                if (st == A2C_ERR_INVALID_ARG) {  // not a schedule of this kernel
                    st = A2C_OK;
                    continue;
                }
                st = part == 0 ? plan_apply_forward_schedule(p, k, w, s, !own_f)
                               : plan_apply_adjoint_schedule(p, k, w, s, !own_b);
                if (st == A2C_ERR_UNSUPPORTED) {  // too many chunks, or staging beyond LDS
                    st = A2C_OK;
                    continue;
                }
                if (st != A2C_OK) break;
                (part == 0 ? own_f : own_b) = true;
                float t = 0.f;
                st = time_part(part, t);
                if (st != A2C_OK) break;
                // a later candidate (more residues per lane or waves) must be
                // 1 % faster to win: exact ties keep the smaller schedule,
                // while a margin as large as the timing noise would favour
                // the smaller schedules (tried first) over better later ones
                float &best = part == 0 ? best_f : best_b;
                if (t < 0.99f * best) {
                    best = t;
                    (part == 0 ? fK : bK) = k;
                    (part == 0 ? fW : bW) = w;
                }
            }
            if (st != A2C_OK) break;
        }
        if (st == A2C_OK && part == 0) {
            st = plan_apply_forward_schedule(p, fK, fW, s, !own_f);
            if (st == A2C_OK) st = a2c_forward(p, A2C_SCAN, d_angles, d_coords, nullptr, s);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != A2C_OK) return st;
    st = plan_apply_adjoint_schedule(p, bK, bW, s, !own_b);
    if (st != A2C_OK) return st;
    cache_store(cache_path, key, fK, fW, bK, bW);
    if (out_K) *out_K = fK;
    if (out_W) *out_W = fW;
    return A2C_OK;
}
