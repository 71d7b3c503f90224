// Internal declarations shared by the host API and the kernel files.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "a2c.h"

namespace a2c {

constexpr int kWave = 64;
constexpr int kMaxWaves = 16;
constexpr int kMaxChunks = 64;        // chunks of 64 W K residues per tile
// dynamic LDS allowed to the full-atom kernels (160 KB per workgroup on
// gfx950, less the static tables)
constexpr int kMaxDynamicLds = 136 * 1024;
// Launch-bound classes of the scan kernels: up to 8 waves per workgroup
// (512 lanes) a kernel may use up to 256 VGPRs without spilling; 16 waves
// cap it at 128.  Launchers pick the class from the schedule's wave count.
constexpr int kLbSmall = 512, kLbLarge = 1024;
// Source of the upstream coordinate gradient in the recompute adjoints: read
// from memory, or 2 (r - t) of the squared distance to a target (the fused
// training step).
constexpr int kGradLoad = 0, kGradMse = 1;
// Window look-back: tagged 64-bit words per tile aggregate (a 3x4 affine)
constexpr int kLbWords = 12;
// LRMSD: atoms per segment (one workgroup of 256 lanes, 16 atoms per lane)
constexpr int kLrSegAtoms = 4096;
// LRMSD gradient pieces: four atoms per thread of a 256-thread workgroup
constexpr int kLrPieceAtoms = 1024;

// Backbone slot constants in float32, slot order N (omega), CA (phi), C (psi).
// (ct, st) is a float32 pair chosen so that ct^2 + st^2 is as close to 1 as
// float32 allows near (cos theta, sin theta), which keeps the repeated fixed
// rotations from drifting in scale along long chains.
struct BBParams {
    float ct[3], st[3], d[3], inv_d[3];
};

// Full-atom constants of one residue type.  Frames: 0 N, 1 CA, 2 C (spine,
// backbone geometry) and 3 + f for side frame f; side frames form a chain
// CA -> 0 -> 1 -> ... (frame f hangs off f-1), frame 0 through a fixed
// rotation about CA's x axis.  Atoms are grouped by frame.
// One atom of a residue type: position in its frame and output slot, packed
// so that a kernel reads it from LDS in one 16-byte access.
struct alignas(16) FAAtom {
    float x, y, z;
    int32_t slot;
};

struct FAType {
    int32_t n_atoms;
    int32_t n_side;
    int32_t side_chi[4];            // 1: torsion chi_{f+1} (plane 3 + f); 0: fixed 0
    float pre_c, pre_s;             // fixed rotation of side frame 0
    float ct[4], st[4], d[4], inv_d[4];
    int32_t fbegin[7], fcount[7];   // atoms of frame k in the sorted lists
    int32_t origin_slot[7];         // residue slot of the atom at frame k's origin
    FAAtom atom[A2C_MAX_RESIDUE_ATOMS];   // sorted by frame
};

struct FATable {
    FAType t[A2C_NUM_RESIDUE_TYPES];
    int32_t max_count[7];           // max atoms per frame over the types
    int32_t max_side;
};

// One scan schedule: K residues per lane, W waves per workgroup, and the
// layouts built for them: tiles (chains of at most one chunk of 64 W K
// residues packed whole into tiles of at most one chunk; a longer chain
// alone) and/or windows of at most one chunk C with a look-back table
// (forwards and the full-atom adjoint: windows only; backbone adjoint: both,
// windows for the adjoint from coordinates, tiles for the recomputing
// adjoint and the fused step).  Windows hold whole chains where every chain
// fits in one, and are fixed, [t C, t C + C), otherwise.  n_tiles counts the
// layout the schedule reports: windows where there are no tiles.
struct Sched {
    int32_t K = 4, W = 4, n_tiles = 0;
    int32_t n_win = 0;                   // windows (0: none)
    int32_t *d_wstart = nullptr;         // n_win + 1 window boundaries (residues)
    bool whole_chains = false;           // every window holds whole chains (no
                                         // window waits on another)
    int32_t *d_look = nullptr;           // n_win: forward, the first window whose
                                         // aggregate window t composes; adjoint, the
                                         // last window whose wrench it adds (t: none)
    uint64_t *d_status = nullptr;        // n_win x kLbWords tagged words
    // full-atom adjoint: a spine pass publishes each window's aggregate in
    // its own tagged words; each window of the adjoint composes those of the
    // windows its first chain spans (from d_look_fwd[t] to t - 1)
    int32_t *d_look_fwd = nullptr;       // n_win, first window to compose
    uint64_t *d_status_fwd = nullptr;    // n_win x kLbWords tagged words
    int32_t fa_stage_atoms = 0;          // per-wave staging (floats per plane)
    bool fa_unstaged = false;            // stage too large for the LDS: direct I/O
    bool multi_chunk = false;            // some tile spans several chunks
    int32_t *d_tile_res = nullptr;       // n_tiles (first, end) residue pairs, longest first
    // fused training step: each tile's share of the loss, and the count of
    // tiles done (the last one sums the shares; it re-arms the count to 0)
    float *d_loss_part = nullptr;        // n_tiles
    uint32_t *d_loss_count = nullptr;    // 1
};

}  // namespace a2c

struct a2c_plan {
    a2c_model model;
    int device = 0;
    int n_cu = 0;                        // compute units of the device
    int32_t n_chains = 0;
    int64_t R = 0, A = 0;
    int32_t max_len = 0;
    std::vector<int32_t> res_off;        // n_chains + 1
    std::vector<int32_t> chain_atom_off; // n_chains + 1
    std::vector<int32_t> res_atom_off;   // R + 1
    std::vector<uint8_t> seq;
    // schedules: fs for the forward, bs for the adjoint and the fused step
    a2c::Sched fs, bs;
    // device tables of schedules that were replaced: a graph captured before
    // the change still launches with them, so they live until the plan does
    std::vector<void *> retired;
    // store-vs-recompute threshold: the forward's coordinates (12 bytes per
    // atom) are kept for the adjoint while they fit; 0 = always recompute
    size_t mem_budget = 0;
    // the adjoints write the angle gradients with non-temporal stores (at
    // least kNtGradBytes of them)
    bool nt_grad = false;
    // device tables
    uint32_t *d_head_bits = nullptr;     // bit r: residue r starts a chain (bit R set)
    int32_t *d_res_off = nullptr;        // chain residue offsets (plain form)
    int32_t *d_res_atom_off = nullptr;   // R + 1 (full-atom)
    uint8_t *d_seq = nullptr;            // R (full-atom)
    a2c::FATable *d_fa = nullptr;        // full-atom constants
    a2c::BBParams bb{};
    a2c::FATable fa_host{};
    // LRMSD segments (the sums): runs of at most kLrSegAtoms atoms of one
    // chain; pieces (the gradient): runs of at most kLrPieceAtoms
    int32_t lr_n_seg = 0;
    std::vector<int32_t> lr_seg_atom;    // lr_n_seg + 1 first atoms (last = A)
    std::vector<int32_t> lr_seg_origin;  // lr_n_seg first atom of each segment's chain
    std::vector<int32_t> lr_chain_seg;   // n_chains + 1 first segment of each chain
    int32_t lr_n_piece = 0;
    std::vector<int32_t> lr_piece_atom;  // lr_n_piece + 1 first atoms (last = A)
    std::vector<int32_t> lr_piece_chain; // lr_n_piece chain of each piece
    int8_t *d_chi_slots = nullptr;       // [20][4][4] chi atom slots (full-atom)
    int32_t *d_lr_seg_atom = nullptr;
    int32_t *d_lr_seg_origin = nullptr;
    int32_t *d_lr_chain_seg = nullptr;
    int32_t *d_lr_piece_atom = nullptr;
    int32_t *d_lr_piece_chain = nullptr;
};

namespace a2c {

// Angle gradients of at least this many bytes are written with non-temporal
// stores: nothing in a training step reads them before the next step, and
// on large batches their cache lines would otherwise evict coordinates and
// upstream gradients that the step reads again.  Below it the cached stores
// are faster (the whole step then stays in the caches).
constexpr size_t kNtGradBytes = (size_t)4 << 20;

void set_error(const std::string &msg);
// the checks a2c_plan_set_schedule (and the adjoint setter) makes on (K, W),
// without the device; the forward setter's checks (K = 8 too for the backbone)
a2c_status check_schedule_args(const a2c_plan *p, int32_t K, int32_t W);
a2c_status check_forward_schedule_args(const a2c_plan *p, int32_t K, int32_t W);
hipError_t launch_fill_zero(float *x, int64_t n, hipStream_t s);
// float32 (cos t, sin t) pair with squared norm closest to 1
void unit_pair(double t, float &c, float &s);
a2c_status hip_fail(hipError_t e, const char *what);

// Launchers (each returns hipSuccess or the launch error)
// quat: the comparison form with the quaternion + translation scan state
hipError_t launch_bb_forward_scan(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s,
                                  bool quat = false);
hipError_t launch_bb_backward_scan(const a2c_plan &p, const float *ang, const float *xyz,
                                   const float *g, float *gang, hipStream_t s);
hipError_t launch_bb_forward_plain(const a2c_plan &p, const float *ang, float *xyz, float *ws,
                                   hipStream_t s);
hipError_t launch_bb_backward_plain(const a2c_plan &p, const float *ang, const float *g,
                                    float *gang, const float *ws, hipStream_t s);
// loss (may be NULL): receives sum |r - t|^2, from the schedule's per-tile
// shares (bs.d_loss_part, bs.d_loss_count)
hipError_t launch_bb_mse_step(const a2c_plan &p, const float *ang, const float *tgt, float *xyz,
                              float *loss, float *gang, hipStream_t s);
hipError_t launch_fa_mse_step(const a2c_plan &p, const float *ang, const float *tgt, float *xyz,
                              float *loss, float *gang, hipStream_t s);
hipError_t launch_fa_forward_scan(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s);
hipError_t launch_fa_backward_scan(const a2c_plan &p, const float *ang, const float *xyz,
                                   const float *g, float *gang, hipStream_t s);
void build_lrmsd_segments(a2c_plan &p);
void build_chi_slots(const FATable &T, int8_t (&out)[A2C_NUM_RESIDUE_TYPES][4][4]);
size_t lrmsd_workspace_bytes(const a2c_plan &p);
// device address of the no-allocation LRMSD scratch on `device` (current)
a2c_status lrmsd_scratch_setup(int device);
void fa_allow_large_lds();
void bb_allow_large_lds();

}  // namespace a2c
