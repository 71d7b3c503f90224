// Host side of the C ABI declared in include/a2c.h: argument validation,
// plan construction (tile packing, head bits, geometry constants, full-atom
// tables) and kernel dispatch.  No call here that can be captured allocates
// or synchronises.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "a2c_internal.h"

namespace a2c {

namespace {
thread_local std::string g_last_error;

a2c_status fail(a2c_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }
bool valid_angle(double v) { return std::isfinite(v) && v > 0.0 && v < 180.0; }

a2c_status upload(void **dst, const void *src, size_t bytes, hipStream_t s)
{
    if (*dst) {
        (void)hipFree(*dst);
        *dst = nullptr;
    }
    if (bytes == 0) return A2C_OK;
    hipError_t e = hipMalloc(dst, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    e = hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    return A2C_OK;
}

void free_sched(Sched &S)
{
    (void)hipFree(S.d_tile_res);
    (void)hipFree(S.d_loss_part);
    (void)hipFree(S.d_loss_count);
    (void)hipFree(S.d_wstart);
    (void)hipFree(S.d_look);
    (void)hipFree(S.d_status);
    (void)hipFree(S.d_look_fwd);
    (void)hipFree(S.d_status_fwd);
    S.d_tile_res = nullptr;
    S.d_loss_part = nullptr;
    S.d_loss_count = nullptr;
    S.d_wstart = nullptr;
    S.d_look = nullptr;
    S.d_status = nullptr;
    S.d_look_fwd = nullptr;
    S.d_status_fwd = nullptr;
}

// Window boundaries for windows of at most `cap` residues (n_win + 1
// entries; none for an empty batch).  Where every chain fits in a window and
// packing whole chains greedily, in order, takes at most 1/8 more windows
// than cutting the batch into fixed windows [t cap, t cap + cap), or no more
// windows than the device has CUs (a launch that leaves CUs idle anyway),
// the windows hold whole chains: no chain crosses a window edge and no window
// waits on another (whole_chains is set).  Otherwise the fixed windows,
// wherever the chains fall.  Zero-length chains take no space.
std::vector<int64_t> window_starts(const a2c_plan *p, int64_t cap, bool &whole_chains)
{
    std::vector<int64_t> st;
    whole_chains = false;
    if (p->R == 0) return st;
    const int64_t n_fixed = (p->R + cap - 1) / cap;
    if (p->max_len <= cap) {
        st.push_back(0);
        int64_t cur = 0;  // residues in the open window
        for (size_t c = 0; c + 1 < p->res_off.size(); ++c) {
            const int64_t L = p->res_off[c + 1] - p->res_off[c];
            if (L == 0) continue;
            if (cur + L > cap) {
                st.push_back(p->res_off[c]);
                cur = 0;
            }
            cur += L;
        }
        st.push_back(p->R);
        const int64_t n_whole = (int64_t)st.size() - 1;
        if (n_whole <= n_fixed + n_fixed / 8 || n_whole <= p->n_cu) {
            whole_chains = true;
            return st;
        }
        st.clear();
    }
    for (int64_t b = 0; b < p->R; b += cap) st.push_back(b);
    st.push_back(p->R);
    return st;
}

// The window holding residue r (starts as from window_starts).
int32_t window_of(const std::vector<int64_t> &starts, int64_t r)
{
    return (int32_t)(std::upper_bound(starts.begin(), starts.end() - 1, r) - starts.begin()) - 1;
}

// Look-back table and tagged words of the windows given by starts.  Forward
// (look_back): for each window t the first window whose aggregate its
// carry-in needs, i.e. the window holding the head of the chain its first
// residue belongs to (t itself when a chain starts there).  Adjoint: the last
// window whose wrench it adds, i.e. the window holding the end of the chain
// of its last residue (t itself when a chain ends there).  The tagged words
// start at tag 0.
a2c_status build_windows(const a2c_plan *p, const std::vector<int64_t> &starts, bool look_back,
                         int32_t *&d_look, uint64_t *&d_status, int32_t &n_win, hipStream_t s)
{
    const int64_t n = starts.empty() ? 0 : (int64_t)starts.size() - 1;
    std::vector<int32_t> look((size_t)n);
    size_t c = 0;  // non-empty chain holding the residue: res_off[c] <= r < res_off[c + 1]
    for (int64_t t = 0; t < n; ++t) {
        const int64_t r = look_back ? starts[(size_t)t] : starts[(size_t)t + 1] - 1;
        while (p->res_off[c + 1] <= r) ++c;
        look[(size_t)t] =
            window_of(starts, look_back ? p->res_off[c] : (int64_t)p->res_off[c + 1] - 1);
    }
    n_win = (int32_t)n;
    a2c_status st = upload((void **)&d_look, look.data(), look.size() * sizeof(int32_t), s);
    if (st != A2C_OK) return st;
    const size_t words = (size_t)std::max<int64_t>(1, n) * kLbWords * sizeof(uint64_t);
    hipError_t e = hipMalloc((void **)&d_status, words);
    if (e == hipSuccess) e = hipMemsetAsync(d_status, 0, words, s);
    if (e != hipSuccess) return hip_fail(e, "look-back words");
    return A2C_OK;
}

// The window boundaries as int32 on the device.
a2c_status upload_starts(const std::vector<int64_t> &starts, int32_t *&d_wstart, hipStream_t s)
{
    std::vector<int32_t> v(starts.begin(), starts.end());
    return upload((void **)&d_wstart, v.data(), v.size() * sizeof(int32_t), s);
}

// Pack the tiles of schedule (K, W) and upload its tile table into out
// (whose own table, if any, the caller frees).
// Greedy packing of whole chains, in order, into tiles: chains of at most one
// chunk (`cap` residues) share tiles of at most `cap` residues; a longer chain
// gets a tile of its own, which the kernels walk chunk by chunk.  Zero-length
// chains produce nothing and never open a tile.
std::vector<int32_t> pack_tiles(const std::vector<int32_t> &off, int64_t cap)
{
    std::vector<int32_t> tiles;
    const size_t n = off.size() - 1;
    int64_t cur = 0;
    tiles.push_back(0);
    for (size_t c = 0; c < n; ++c) {
        const int64_t L = off[c + 1] - off[c];
        if (L == 0) continue;
        if (cur > 0 && (cur + L > cap || L > cap)) {
            tiles.push_back(off[c]);
            cur = 0;
        }
        cur += L;
        if (L > cap) {  // a long chain closes its own tile
            tiles.push_back(off[c + 1]);
            cur = 0;
        }
    }
    if (cur > 0) tiles.push_back(off[n]);
    if (tiles.size() == 1) tiles.clear();  // no residues
    return tiles;
}

// Layouts of a schedule (see Sched).
enum SchedRole { kRoleForward, kRoleAdjoint };

a2c_status build_sched(const a2c_plan *p, int32_t K, int32_t W, Sched &out, hipStream_t s,
                       SchedRole role)
{
    const bool flat = role == kRoleForward || p->model == A2C_FULLATOM;  // windows only
    const bool windows = flat || p->model == A2C_BACKBONE;
    const int64_t cap = (int64_t)kWave * W * K;  // residues per chunk
    if (p->max_len > cap * kMaxChunks)
        return fail(A2C_ERR_UNSUPPORTED, "a chain of " + std::to_string(p->max_len) +
                                             " residues needs more than " +
                                             std::to_string(kMaxChunks) + " chunks of " +
                                             std::to_string(cap) + " residues");
    bool whole_chains = false;
    const std::vector<int64_t> starts =
        windows ? window_starts(p, cap, whole_chains) : std::vector<int64_t>();
    if (flat) {
        Sched S;
        S.K = K;
        S.W = W;
        S.whole_chains = whole_chains;
        if (p->model == A2C_FULLATOM) {
            // per-wave LDS stage of three planes (the adjoint from
            // coordinates stages six where they fit): the most atoms of one
            // wave's run of 64 K residues
            int64_t most = 1;
            for (size_t t = 0; t + 1 < starts.size(); ++t)
                for (int64_t rb = starts[t]; rb < starts[t + 1]; rb += (int64_t)kWave * K) {
                    const int64_t re = std::min<int64_t>(rb + (int64_t)kWave * K, starts[t + 1]);
                    most = std::max<int64_t>(most, p->res_atom_off[re] - p->res_atom_off[rb]);
                }
            if ((size_t)W * 3 * most * sizeof(float) > (size_t)kMaxDynamicLds)
                S.fa_unstaged = true;  // atoms straight to global memory
            else
                S.fa_stage_atoms = (int32_t)most;
        }
        const bool fwd = role == kRoleForward;
        a2c_status st = upload_starts(starts, S.d_wstart, s);
        if (st == A2C_OK) st = build_windows(p, starts, fwd, S.d_look, S.d_status, S.n_win, s);
        S.n_tiles = S.n_win;
        if (st == A2C_OK && !fwd) {
            // the full-atom adjoint: the spine pass's words and the windows
            // whose aggregates each window composes (the fused step's loss
            // shares travel in the adjoint's own tagged words)
            int32_t n2 = 0;
            st = build_windows(p, starts, true, S.d_look_fwd, S.d_status_fwd, n2, s);
        }
        if (st == A2C_OK) {
            const hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
        }
        if (st != A2C_OK) {
            free_sched(S);
            return st;
        }
        out = S;
        return A2C_OK;
    }
    std::vector<int32_t> tiles = pack_tiles(p->res_off, cap);
    int32_t stage_atoms = 0;
    if (p->model == A2C_FULLATOM) {
        // largest atom run of one wave in one chunk: the per-wave staging size
        const int64_t per_wave = (int64_t)kWave * K;
        for (size_t t = 0; t + 1 < tiles.size(); ++t)
            for (int64_t cs = tiles[t]; cs < tiles[t + 1]; cs += cap) {
                const int64_t ce = std::min<int64_t>(cs + cap, tiles[t + 1]);
                for (int64_t rb = cs; rb < ce; rb += per_wave) {
                    const int64_t re = std::min<int64_t>(rb + per_wave, ce);
                    stage_atoms = std::max<int32_t>(
                        stage_atoms, p->res_atom_off[re] - p->res_atom_off[rb]);
                }
            }
        stage_atoms = std::max<int32_t>(stage_atoms, 1);
    }
    // full-atom atom I/O goes through a per-wave LDS stage of three planes
    // (forward, recompute adjoint; the coordinate-mode adjoint stages six and
    // uses the recompute form where they do not fit); where three planes do
    // not fit either, the kernels read and write the atoms in global memory
    // directly
    bool unstaged = false;
    if (p->model == A2C_FULLATOM &&
        (size_t)W * 3 * stage_atoms * sizeof(float) > (size_t)kMaxDynamicLds) {
        unstaged = true;
        stage_atoms = 0;
    }
    Sched S;
    S.whole_chains = whole_chains;
    S.fa_stage_atoms = stage_atoms;
    S.fa_unstaged = unstaged;
    S.multi_chunk = false;
    for (size_t t = 0; t + 1 < tiles.size(); ++t)
        if (tiles[t + 1] - tiles[t] > cap) S.multi_chunk = true;
    S.K = K;
    S.W = W;
    S.n_tiles = tiles.empty() ? 0 : (int32_t)tiles.size() - 1;
    // (first, end) residue pairs, longest tile first: tiles are independent,
    // and dispatching the long ones (multi-chunk chains, full tiles) first
    // keeps them out of the tail of the launch
    std::vector<int32_t> order(S.n_tiles);
    for (int32_t t = 0; t < S.n_tiles; ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return tiles[a + 1] - tiles[a] > tiles[b + 1] - tiles[b];
    });
    std::vector<int32_t> pairs(2 * (size_t)S.n_tiles);
    for (int32_t t = 0; t < S.n_tiles; ++t) {
        pairs[2 * t] = tiles[order[t]];
        pairs[2 * t + 1] = tiles[order[t] + 1];
    }
    a2c_status st = upload((void **)&S.d_tile_res, pairs.data(), pairs.size() * sizeof(int32_t), s);
    if (st == A2C_OK && windows) st = upload_starts(starts, S.d_wstart, s);
    if (st == A2C_OK && windows) st = build_windows(p, starts, false, S.d_look, S.d_status, S.n_win, s);
    // the fused step's per-tile loss shares and its count of finished tiles
    // (zero: the last tile of every launch sets it back to zero)
    if (st == A2C_OK) {
        hipError_t e = hipMalloc((void **)&S.d_loss_part,
                                 std::max<size_t>(1, S.n_tiles) * sizeof(float));
        if (e == hipSuccess) e = hipMalloc((void **)&S.d_loss_count, sizeof(uint32_t));
        if (e == hipSuccess) e = hipMemsetAsync(S.d_loss_count, 0, sizeof(uint32_t), s);
        if (e != hipSuccess) st = hip_fail(e, "loss scratch");
    }
    if (st == A2C_OK) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    }
    if (st != A2C_OK) {
        free_sched(S);
        return st;
    }
    out = S;
    return A2C_OK;
}

// A replaced schedule's device tables stay allocated until the plan is
// destroyed: a graph captured before the change still launches with them.
void retire_sched(a2c_plan *p, Sched &S)
{
    for (void *q : {(void *)S.d_tile_res, (void *)S.d_loss_part, (void *)S.d_loss_count,
                    (void *)S.d_wstart, (void *)S.d_look, (void *)S.d_status,
                    (void *)S.d_look_fwd, (void *)S.d_status_fwd})
        if (q) p->retired.push_back(q);
    S.d_tile_res = nullptr;
    S.d_loss_part = nullptr;
    S.d_loss_count = nullptr;
    S.d_wstart = nullptr;
    S.d_look = nullptr;
    S.d_status = nullptr;
    S.d_look_fwd = nullptr;
    S.d_status_fwd = nullptr;
}

// Replace one of the plan's schedules; on failure it stays as it was.  The
// old tables are retired (kept until the plan is destroyed), or freed at once
// when retire_old is false: the autotuner's own candidates, which no graph
// can have captured.
a2c_status set_sched(a2c_plan *p, Sched &dst, int32_t K, int32_t W, hipStream_t s,
                     bool retire_old = true)
{
    Sched S;
    const a2c_status st = build_sched(p, K, W, S, s, &dst == &p->fs ? kRoleForward : kRoleAdjoint);
    if (st != A2C_OK) return st;
    if (retire_old) retire_sched(p, dst);
    else free_sched(dst);
    dst = S;
    return A2C_OK;
}

// Both schedules (forward, and adjoint / fused step) to (K, W).
a2c_status apply_schedule(a2c_plan *p, int32_t K, int32_t W, hipStream_t s,
                          bool retire_old = true)
{
    Sched f, b;
    a2c_status st = build_sched(p, K, W, f, s, kRoleForward);
    if (st != A2C_OK) return st;
    st = build_sched(p, K, W, b, s, kRoleAdjoint);
    if (st != A2C_OK) {
        free_sched(f);
        return st;
    }
    if (retire_old) {
        retire_sched(p, p->fs);
        retire_sched(p, p->bs);
    } else {
        free_sched(p->fs);
        free_sched(p->bs);
    }
    p->fs = f;
    p->bs = b;
    return A2C_OK;
}

// One chunk per chain where a 16-wave chunk holds it; full-atom keeps four
// waves so the per-wave atom staging stays small, and widens the chunk only
// when its longest chain would need more than kMaxChunks chunks.
void default_schedule(const a2c_plan &p, int32_t &K, int32_t &W)
{
    K = p.model == A2C_BACKBONE ? 4 : 1;
    const int64_t per_wave = (int64_t)kWave * K;
    const int64_t wmax = p.model == A2C_BACKBONE ? kMaxWaves : 4;
    W = (int32_t)std::min<int64_t>(wmax, std::max<int64_t>(1, (p.max_len + per_wave - 1) / per_wave));
    while ((int64_t)p.max_len > (int64_t)kWave * W * K * kMaxChunks) {
        if (W < kMaxWaves) W = std::min<int32_t>(kMaxWaves, 2 * W);
        else if (K < 2) K = 2;
        else break;  // plan_create has already rejected longer chains
    }
}

bool check_device(const a2c_plan *p)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    return dev == p->device;
}

}  // namespace

// The float32 (c, s) pair within +-2 ulps of (cos t, sin t) whose squared
// norm is closest to 1 (ties broken by the angle error).  Independent
// rounding of cos and sin leaves c^2 + s^2 - 1 ~ 1e-7, a scale error that
// every residue repeats; the pair search makes it ~1e-9.
void unit_pair(double t, float &c_out, float &s_out)
{
    const float c0 = (float)std::cos(t), s0 = (float)std::sin(t);
    double best = std::numeric_limits<double>::infinity();
    c_out = c0;
    s_out = s0;
    float cs[5], ss[5];
    cs[2] = c0;
    ss[2] = s0;
    cs[3] = std::nextafter(c0, 2.f); cs[4] = std::nextafter(cs[3], 2.f);
    cs[1] = std::nextafter(c0, -2.f); cs[0] = std::nextafter(cs[1], -2.f);
    ss[3] = std::nextafter(s0, 2.f); ss[4] = std::nextafter(ss[3], 2.f);
    ss[1] = std::nextafter(s0, -2.f); ss[0] = std::nextafter(ss[1], -2.f);
    for (float c : cs)
        for (float s : ss) {
            const double e = std::fabs((double)c * c + (double)s * s - 1.0) +
                             1e-3 * std::fabs(std::atan2((double)s, (double)c) - t);
            if (e < best) {
                best = e;
                c_out = c;
                s_out = s;
            }
        }
}

// The forward setter's checks: the backbone forward also takes K = 8.
a2c_status check_forward_schedule_args(const a2c_plan *p, int32_t K, int32_t W)
{
    if (p->model == A2C_BACKBONE && K == 8) {
        if (W < 1 || W > kMaxWaves) return fail(A2C_ERR_INVALID_ARG, "waves_per_group must be 1..16");
        return A2C_OK;
    }
    return check_schedule_args(p, K, W);
}

// The checks a2c_plan_set_schedule makes on (K, W), without the device.
a2c_status check_schedule_args(const a2c_plan *p, int32_t K, int32_t W)
{
    if (!(K == 1 || K == 2 || K == 4))
        return fail(A2C_ERR_INVALID_ARG, "res_per_lane must be 1, 2 or 4");
    if (p->model == A2C_FULLATOM && K == 4)
        return fail(A2C_ERR_INVALID_ARG, "the full-atom kernels take res_per_lane 1 or 2");
    if (W < 1 || W > kMaxWaves) return fail(A2C_ERR_INVALID_ARG, "waves_per_group must be 1..16");
    return A2C_OK;
}

namespace {
__global__ void fill_zero_kernel(float *x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.f;
}
}  // namespace

// A kernel, not hipMemsetAsync: callers may capture it in a graph.
hipError_t launch_fill_zero(float *x, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

void set_error(const std::string &msg) { g_last_error = msg; }

a2c_status hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return A2C_ERR_HIP;
}

a2c_status build_fullatom_tables(a2c_plan *p, const a2c_residue_table *table);

a2c_status plan_apply_adjoint_schedule(a2c_plan *p, int32_t K, int32_t W, hipStream_t s,
                                       bool retire_old)
{
    return set_sched(p, p->bs, K, W, s, retire_old);
}

a2c_status plan_apply_forward_schedule(a2c_plan *p, int32_t K, int32_t W, hipStream_t s,
                                       bool retire_old)
{
    return set_sched(p, p->fs, K, W, s, retire_old);
}

}  // namespace a2c

using namespace a2c;

extern "C" {

const char *a2c_version(void) { return "a2c 0.1 gfx950"; }

const char *a2c_status_string(int32_t st)
{
    switch (st) {
    case A2C_OK: return "ok";
    case A2C_ERR_INVALID_ARG: return "invalid argument";
    case A2C_ERR_UNSUPPORTED: return "unsupported";
    case A2C_ERR_WORKSPACE: return "workspace missing or too small";
    case A2C_ERR_HIP: return "HIP runtime error";
    case A2C_ERR_STATE: return "invalid state";
    }
    return "unknown status";
}

const char *a2c_last_error(void) { return g_last_error.c_str(); }

void a2c_plan_destroy(a2c_plan *p)
{
    if (!p) return;
    free_sched(p->fs);
    free_sched(p->bs);
    for (void *q : p->retired) (void)hipFree(q);
    (void)hipFree(p->d_head_bits);
    (void)hipFree(p->d_res_off);
    (void)hipFree(p->d_res_atom_off);
    (void)hipFree(p->d_seq);
    (void)hipFree(p->d_fa);
    (void)hipFree(p->d_chi_slots);
    (void)hipFree(p->d_lr_seg_atom);
    (void)hipFree(p->d_lr_seg_origin);
    (void)hipFree(p->d_lr_chain_seg);
    (void)hipFree(p->d_lr_piece_atom);
    (void)hipFree(p->d_lr_piece_chain);
    delete p;
}

a2c_status a2c_plan_create(a2c_plan **out, int32_t model_id, int32_t n_chains,
                           const int32_t *h_res_offsets, const uint8_t *h_seq,
                           const a2c_backbone_geometry *geom, const a2c_residue_table *table,
                           size_t mem_budget_bytes, void *stream)
{
    if (!out) return fail(A2C_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (model_id != A2C_BACKBONE && model_id != A2C_FULLATOM)
        return fail(A2C_ERR_INVALID_ARG, "unknown model");
    const a2c_model model = (a2c_model)model_id;
    if (n_chains < 0) return fail(A2C_ERR_INVALID_ARG, "n_chains < 0");
    if (!h_res_offsets) return fail(A2C_ERR_INVALID_ARG, "h_res_offsets is NULL");
    if (h_res_offsets[0] != 0) return fail(A2C_ERR_INVALID_ARG, "h_res_offsets[0] != 0");
    int32_t max_len = 0;
    for (int32_t c = 0; c < n_chains; ++c) {
        const int64_t L = (int64_t)h_res_offsets[c + 1] - h_res_offsets[c];
        if (L < 0)
            return fail(A2C_ERR_INVALID_ARG,
                        "h_res_offsets decreases at chain " + std::to_string(c));
        max_len = std::max<int32_t>(max_len, (int32_t)L);
    }
    const int64_t R = h_res_offsets[n_chains];
    if (R > (int64_t)std::numeric_limits<int32_t>::max() / 16)
        return fail(A2C_ERR_UNSUPPORTED, "too many residues for int32 atom offsets");
    const int32_t max_tile = kMaxChunks * kWave * kMaxWaves * (model == A2C_BACKBONE ? 4 : 2);
    if (max_len > max_tile)
        return fail(A2C_ERR_UNSUPPORTED, "chain longer than " + std::to_string(max_tile) +
                                             " residues");
    if (model == A2C_FULLATOM) {
        if (!table) return fail(A2C_ERR_INVALID_ARG, "full-atom plan needs a residue table");
        if (R > 0 && !h_seq) return fail(A2C_ERR_INVALID_ARG, "full-atom plan needs h_seq");
        for (int64_t r = 0; r < R; ++r)
            if (h_seq[r] >= A2C_NUM_RESIDUE_TYPES)
                return fail(A2C_ERR_INVALID_ARG, "residue code " + std::to_string(h_seq[r]) +
                                                     " >= 20 at residue " + std::to_string(r));
    }
    a2c_backbone_geometry g = {1.458, 1.525, 1.329, 111.2, 116.2, 121.7};
    if (geom) g = *geom;
    if (!finite_pos(g.bond_n_ca) || !finite_pos(g.bond_ca_c) || !finite_pos(g.bond_c_n) ||
        !valid_angle(g.angle_n_ca_c) || !valid_angle(g.angle_ca_c_n) ||
        !valid_angle(g.angle_c_n_ca))
        return fail(A2C_ERR_INVALID_ARG, "backbone geometry out of range");

    hipStream_t s = (hipStream_t)stream;
    a2c_plan *p = new a2c_plan();
    p->model = model;
    p->n_chains = n_chains;
    p->R = R;
    p->max_len = max_len;
    p->mem_budget = mem_budget_bytes;
    p->res_off.assign(h_res_offsets, h_res_offsets + n_chains + 1);
    // slot constants (N, CA, C): bond to the previous atom and the bond angle
    // at the previous atom; theta = pi - angle
    const double pi = 3.14159265358979323846;
    const double bond[3] = {g.bond_c_n, g.bond_n_ca, g.bond_ca_c};
    const double angle[3] = {g.angle_ca_c_n, g.angle_c_n_ca, g.angle_n_ca_c};
    for (int k = 0; k < 3; ++k) {
        unit_pair(pi - angle[k] * (pi / 180.0), p->bb.ct[k], p->bb.st[k]);
        p->bb.d[k] = (float)bond[k];
        p->bb.inv_d[k] = (float)(1.0 / bond[k]);
    }

    a2c_status st = A2C_OK;
    if (model == A2C_BACKBONE) {
        p->A = 3 * R;
        p->chain_atom_off.resize(n_chains + 1);
        for (int32_t c = 0; c <= n_chains; ++c) p->chain_atom_off[c] = 3 * h_res_offsets[c];
    } else {
        p->seq.assign(h_seq, h_seq + R);
        st = build_fullatom_tables(p, table);
        if (st != A2C_OK) {
            a2c_plan_destroy(p);
            return st;
        }
    }
    p->nt_grad = (size_t)R * (model == A2C_BACKBONE ? 3 : 7) * sizeof(float) >= kNtGradBytes;
    // host tables are complete: now the device
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        a2c_plan_destroy(p);
        return hip_fail(e, "hipGetDevice");
    }
    p->device = dev;
    e = hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) {
        a2c_plan_destroy(p);
        return hip_fail(e, "hipDeviceGetAttribute");
    }
    // chain-head bits, padded by two words so a lane may read one word past
    std::vector<uint32_t> bits((size_t)((R + 64) / 32 + 2), 0u);
    for (int32_t c = 0; c < n_chains; ++c)
        if (h_res_offsets[c + 1] > h_res_offsets[c])
            bits[h_res_offsets[c] >> 5] |= 1u << (h_res_offsets[c] & 31);
    bits[R >> 5] |= 1u << (R & 31);
    st = upload((void **)&p->d_head_bits, bits.data(), bits.size() * sizeof(uint32_t), s);
    if (st == A2C_OK)
        st = upload((void **)&p->d_res_off, p->res_off.data(), p->res_off.size() * sizeof(int32_t), s);
    if (st == A2C_OK && model == A2C_FULLATOM) {
        st = upload((void **)&p->d_res_atom_off, p->res_atom_off.data(),
                    p->res_atom_off.size() * sizeof(int32_t), s);
        if (st == A2C_OK) st = upload((void **)&p->d_seq, p->seq.data(), p->seq.size(), s);
        if (st == A2C_OK) st = upload((void **)&p->d_fa, &p->fa_host, sizeof(FATable), s);
        if (st == A2C_OK) {
            int8_t chi[A2C_NUM_RESIDUE_TYPES][4][4];
            build_chi_slots(p->fa_host, chi);
            st = upload((void **)&p->d_chi_slots, chi, sizeof(chi), s);
        }
    }
    if (st == A2C_OK) {
        build_lrmsd_segments(*p);
        st = upload((void **)&p->d_lr_seg_atom, p->lr_seg_atom.data(),
                    p->lr_seg_atom.size() * sizeof(int32_t), s);
        if (st == A2C_OK)
            st = upload((void **)&p->d_lr_seg_origin, p->lr_seg_origin.data(),
                        p->lr_seg_origin.size() * sizeof(int32_t), s);
        if (st == A2C_OK)
            st = upload((void **)&p->d_lr_chain_seg, p->lr_chain_seg.data(),
                        p->lr_chain_seg.size() * sizeof(int32_t), s);
        if (st == A2C_OK)
            st = upload((void **)&p->d_lr_piece_atom, p->lr_piece_atom.data(),
                        p->lr_piece_atom.size() * sizeof(int32_t), s);
        if (st == A2C_OK)
            st = upload((void **)&p->d_lr_piece_chain, p->lr_piece_chain.data(),
                        p->lr_piece_chain.size() * sizeof(int32_t), s);
    }
    if (st == A2C_OK) st = lrmsd_scratch_setup(dev);
    if (st == A2C_OK) {
        if (model == A2C_FULLATOM) fa_allow_large_lds();
        else bb_allow_large_lds();
    }
    if (st == A2C_OK) {
        int32_t K, W;
        default_schedule(*p, K, W);
        st = apply_schedule(p, K, W, s);
    }
    if (st != A2C_OK) {
        a2c_plan_destroy(p);
        return st;
    }
    *out = p;
    return A2C_OK;
}

a2c_status a2c_plan_sizes(const a2c_plan *p, int64_t *n_res, int64_t *n_atoms)
{
    if (!p) return fail(A2C_ERR_INVALID_ARG, "plan is NULL");
    if (n_res) *n_res = p->R;
    if (n_atoms) *n_atoms = p->A;
    return A2C_OK;
}

a2c_status a2c_plan_atom_offsets(const a2c_plan *p, int32_t *h_chain_atom_offsets,
                                 int32_t *h_res_atom_offsets)
{
    if (!p) return fail(A2C_ERR_INVALID_ARG, "plan is NULL");
    if (h_chain_atom_offsets)
        std::memcpy(h_chain_atom_offsets, p->chain_atom_off.data(),
                    p->chain_atom_off.size() * sizeof(int32_t));
    if (h_res_atom_offsets) {
        if (p->model == A2C_BACKBONE)
            for (int64_t r = 0; r <= p->R; ++r) h_res_atom_offsets[r] = (int32_t)(3 * r);
        else
            std::memcpy(h_res_atom_offsets, p->res_atom_off.data(),
                        p->res_atom_off.size() * sizeof(int32_t));
    }
    return A2C_OK;
}

a2c_status a2c_plan_keep_coords(const a2c_plan *p, int32_t *keep)
{
    if (!p || !keep) return fail(A2C_ERR_INVALID_ARG, "plan or keep is NULL");
    *keep = (uint64_t)p->A * 3 * sizeof(float) <= (uint64_t)p->mem_budget && p->mem_budget > 0
                ? 1 : 0;
    return A2C_OK;
}

a2c_status a2c_plan_workspace_bytes(const a2c_plan *p, int32_t v, size_t *bytes)
{
    if (!p || !bytes) return fail(A2C_ERR_INVALID_ARG, "plan or bytes is NULL");
    if (v == A2C_SCAN || v == A2C_SCAN_QUAT) *bytes = 0;
    else if (v == A2C_PLAIN) *bytes = (size_t)p->A * 12 * sizeof(float);
    else return fail(A2C_ERR_INVALID_ARG, "unknown variant");
    return A2C_OK;
}

a2c_status a2c_plan_set_schedule(a2c_plan *p, int32_t K, int32_t W, void *stream)
{
    if (!p) return fail(A2C_ERR_INVALID_ARG, "plan is NULL");
    const a2c_status sa = check_schedule_args(p, K, W);
    if (sa != A2C_OK) return sa;
    if (!check_device(p)) return fail(A2C_ERR_STATE, "current device is not the plan's device");
    return apply_schedule(p, K, W, (hipStream_t)stream);
}

a2c_status a2c_plan_set_adjoint_schedule(a2c_plan *p, int32_t K, int32_t W, void *stream)
{
    if (!p) return fail(A2C_ERR_INVALID_ARG, "plan is NULL");
    const a2c_status sa = check_schedule_args(p, K, W);
    if (sa != A2C_OK) return sa;
    if (!check_device(p)) return fail(A2C_ERR_STATE, "current device is not the plan's device");
    return set_sched(p, p->bs, K, W, (hipStream_t)stream);
}

a2c_status a2c_plan_set_forward_schedule(a2c_plan *p, int32_t K, int32_t W, void *stream)
{
    if (!p) return fail(A2C_ERR_INVALID_ARG, "plan is NULL");
    const a2c_status sa = check_forward_schedule_args(p, K, W);
    if (sa != A2C_OK) return sa;
    if (!check_device(p)) return fail(A2C_ERR_STATE, "current device is not the plan's device");
    return set_sched(p, p->fs, K, W, (hipStream_t)stream);
}

a2c_status a2c_plan_get_schedule(const a2c_plan *p, int32_t *K, int32_t *W, int32_t *n_tiles)
{
    if (!p) return fail(A2C_ERR_INVALID_ARG, "plan is NULL");
    if (K) *K = p->fs.K;
    if (W) *W = p->fs.W;
    if (n_tiles) *n_tiles = p->fs.n_tiles;
    return A2C_OK;
}

a2c_status a2c_plan_get_adjoint_schedule(const a2c_plan *p, int32_t *K, int32_t *W,
                                         int32_t *n_tiles)
{
    if (!p) return fail(A2C_ERR_INVALID_ARG, "plan is NULL");
    if (K) *K = p->bs.K;
    if (W) *W = p->bs.W;
    if (n_tiles) *n_tiles = p->bs.n_tiles;
    return A2C_OK;
}

a2c_status a2c_forward(a2c_plan *p, int32_t v, const float *d_angles, float *d_coords,
                       void *d_workspace, void *stream)
{
    if (!p) return fail(A2C_ERR_INVALID_ARG, "plan is NULL");
    if (v != A2C_SCAN && v != A2C_PLAIN && v != A2C_SCAN_QUAT)
        return fail(A2C_ERR_INVALID_ARG, "unknown variant");
    if (v == A2C_PLAIN && p->model != A2C_BACKBONE)
        return fail(A2C_ERR_UNSUPPORTED, "the plain form is the backbone comparison only");
    if (v == A2C_SCAN_QUAT && p->model != A2C_BACKBONE)
        return fail(A2C_ERR_UNSUPPORTED, "the quaternion scan state is a backbone comparison only");
    if (p->R == 0) return A2C_OK;
    if (!d_angles || !d_coords) return fail(A2C_ERR_INVALID_ARG, "NULL angles or coords");
    if (v == A2C_PLAIN && !d_workspace)
        return fail(A2C_ERR_WORKSPACE, "the plain form stores M_i in the workspace");
    if (!check_device(p)) return fail(A2C_ERR_STATE, "current device is not the plan's device");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (v == A2C_PLAIN) e = launch_bb_forward_plain(*p, d_angles, d_coords, (float *)d_workspace, s);
    else if (p->model == A2C_BACKBONE)
        e = launch_bb_forward_scan(*p, d_angles, d_coords, s, v == A2C_SCAN_QUAT);
    else e = launch_fa_forward_scan(*p, d_angles, d_coords, s);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return A2C_OK;
}

a2c_status a2c_backward(a2c_plan *p, int32_t v, const float *d_angles, const float *d_coords,
                        const float *d_grad_coords, float *d_grad_angles, void *d_workspace,
                        void *stream)
{
    if (!p) return fail(A2C_ERR_INVALID_ARG, "plan is NULL");
    if (v == A2C_SCAN_QUAT)
        return fail(A2C_ERR_UNSUPPORTED, "the quaternion scan state is a forward comparison only");
    if (v != A2C_SCAN && v != A2C_PLAIN) return fail(A2C_ERR_INVALID_ARG, "unknown variant");
    if (v == A2C_PLAIN && p->model != A2C_BACKBONE)
        return fail(A2C_ERR_UNSUPPORTED, "the plain form is the backbone comparison only");
    if (p->R == 0) return A2C_OK;
    if (!d_grad_coords || !d_grad_angles)
        return fail(A2C_ERR_INVALID_ARG, "NULL grad_coords or grad_angles");
    if (!d_angles) return fail(A2C_ERR_INVALID_ARG, "NULL angles");
    if (v == A2C_PLAIN && !d_workspace)
        return fail(A2C_ERR_WORKSPACE, "the plain backward reads the M_i its forward stored");
    if (!check_device(p)) return fail(A2C_ERR_STATE, "current device is not the plan's device");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (v == A2C_PLAIN)
        e = launch_bb_backward_plain(*p, d_angles, d_grad_coords, d_grad_angles,
                                     (const float *)d_workspace, s);
    else if (p->model == A2C_BACKBONE)
        e = launch_bb_backward_scan(*p, d_angles, d_coords, d_grad_coords, d_grad_angles, s);
    else
        e = launch_fa_backward_scan(*p, d_angles, d_coords, d_grad_coords, d_grad_angles, s);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return A2C_OK;
}

a2c_status a2c_mse_step(a2c_plan *p, const float *d_angles, const float *d_target,
                        float *d_coords, float *d_loss, float *d_grad_angles, void *stream)
{
    if (!p) return fail(A2C_ERR_INVALID_ARG, "plan is NULL");
    if (p->R == 0) {  // the loss of an empty batch is 0 (one fill kernel, capturable)
        if (!d_loss) return A2C_OK;
        if (!check_device(p)) return fail(A2C_ERR_STATE, "current device is not the plan's device");
        const hipError_t e = launch_fill_zero(d_loss, 1, (hipStream_t)stream);
        return e == hipSuccess ? A2C_OK : hip_fail(e, "loss fill launch");
    }
    if (!d_angles || !d_target || !d_grad_angles)
        return fail(A2C_ERR_INVALID_ARG, "NULL angles, target or grad_angles");
    if (!check_device(p)) return fail(A2C_ERR_STATE, "current device is not the plan's device");
    hipStream_t s = (hipStream_t)stream;
    const hipError_t e =
        p->model == A2C_BACKBONE
            ? launch_bb_mse_step(*p, d_angles, d_target, d_coords, d_loss, d_grad_angles, s)
            : launch_fa_mse_step(*p, d_angles, d_target, d_coords, d_loss, d_grad_angles, s);
    if (e != hipSuccess) return hip_fail(e, "training step launch");
    return A2C_OK;
}

}  // extern "C"
