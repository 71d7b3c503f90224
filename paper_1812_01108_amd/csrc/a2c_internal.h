// Internal declarations shared by the host API and the kernel files.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/a2c.h"

namespace a2c {

constexpr int kWave = 64;
constexpr int kMaxWaves = 16;
constexpr int kMaxTileResidues = kWave * kMaxWaves * 4;  // 4096

// Backbone slot constants in float32, slot order N (omega), CA (phi), C (psi).
// (ct, st) is a float32 pair chosen so that ct^2 + st^2 is as close to 1 as
// float32 allows near (cos theta, sin theta), which keeps the repeated fixed
// rotations from drifting in scale along long chains.
struct BBParams {
    float ct[3], st[3], d[3], inv_d[3];
};

// Full-atom constants (device memory, one block per residue type).
struct FAResidue {
    int32_t n_atoms;
    int32_t n_side;
    int32_t side_parent[4];     // 1 = CA frame, 3.. side frames
    int32_t side_plane[4];      // angle plane, or -1 for a fixed torsion of 0
    float side_pre_c[4], side_pre_s[4];  // fixed pre-rotation about x
    float side_ct[4], side_st[4], side_d[4];
    int32_t atom_frame[14];
    float atom_x[14], atom_y[14], atom_z[14];
};

struct FATable {
    FAResidue res[A2C_NUM_RESIDUE_TYPES];
};

}  // namespace a2c

struct a2c_plan {
    a2c_model model;
    int device = 0;
    int32_t n_chains = 0;
    int64_t R = 0, A = 0;
    int32_t max_len = 0;
    std::vector<int32_t> res_off;        // n_chains + 1
    std::vector<int32_t> chain_atom_off; // n_chains + 1
    std::vector<int32_t> res_atom_off;   // R + 1
    std::vector<uint8_t> seq;
    // schedule
    int32_t K = 4, W = 4, n_tiles = 0;
    // device tables
    int32_t *d_tile_res = nullptr;       // n_tiles + 1 residue offsets of tiles
    uint32_t *d_head_bits = nullptr;     // bit r: residue r starts a chain (bit R set)
    int32_t *d_res_off = nullptr;        // chain residue offsets (plain form)
    int32_t *d_res_atom_off = nullptr;   // R + 1 (full-atom)
    uint8_t *d_seq = nullptr;            // R (full-atom)
    a2c::FATable *d_fa = nullptr;        // full-atom constants
    a2c::BBParams bb{};
    a2c::FATable fa_host{};
};

namespace a2c {

void set_error(const std::string &msg);
a2c_status hip_fail(hipError_t e, const char *what);

// Launchers (each returns hipSuccess or the launch error)
hipError_t launch_bb_forward_scan(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s);
hipError_t launch_bb_backward_scan(const a2c_plan &p, const float *ang, const float *xyz,
                                   const float *g, float *gang, hipStream_t s);
hipError_t launch_bb_forward_plain(const a2c_plan &p, const float *ang, float *xyz, float *ws,
                                   hipStream_t s);
hipError_t launch_bb_backward_plain(const a2c_plan &p, const float *ang, const float *g,
                                    float *gang, const float *ws, hipStream_t s);
hipError_t launch_fa_forward_scan(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s);
hipError_t launch_fa_backward_scan(const a2c_plan &p, const float *ang, const float *xyz,
                                   const float *g, float *gang, hipStream_t s);

}  // namespace a2c
