// Internal data layout shared by the host runtime and the gfx950 kernels.
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace fsi {

constexpr int Q = 9;
constexpr int NPOP = 18;            // f_0..f_8 then g_0..g_8
constexpr int TILE_X = 32;          // nodes along i per tile (default shape)
constexpr int TILE_Y = 16;          // nodes along j per tile (default shape)
// tile shapes of the fused kernel (the batch autotuner chooses among them;
// C-grid launches use shape 0)
// (one thread per arrival node: 512-thread workgroups, 256 for 16 x 16)
constexpr int N_TILE_SHAPES = 4;
constexpr int TILE_SHAPES[N_TILE_SHAPES][2] = {{32, 16}, {64, 8}, {16, 32}, {16, 16}};
constexpr int HIST_CAP = 1 << 16;   // force / displacement history records kept

// error bits of the device error word
constexpr unsigned ERR_CFL = 1u;    // departure point outside the node's cells
constexpr unsigned ERR_STATE = 2u;  // rho<=0, T<=0, T>=1, Phi_0<=0, NaN
constexpr unsigned ERR_MESH = 4u;   // det(dx/dxi) <= 0 after blending

enum Dof { DOF_PRESCRIBED = 0, DOF_HEAVE = 1, DOF_PITCH_PLUNGE = 2, DOF_FIXED = 3 };

// Constant description of the (single) body of an instance.
struct Body {
    int dof;
    int present;
    double m, S_a, I_a, k_h, k_a;
    double cx, cy;            // blending centre (undeformed frame)
    double ex, ey;            // elastic axis / rotation centre (undeformed frame)
    double r_rigid, inv_width;// 1 / (r_blend - r_rigid)
    double heave_amp, heave_omega, pitch_amp, pitch_omega;
    double release_time;      // > 0: prescribed motion until then (1DOF / 2DOF)
    int blend_mode;           // 0: radial from (cx, cy); 1: per-node wall distance
    int pad;
};

// Body state at one time level, plus the rotation terms the kernels need.
struct BodySlot {
    double h, a, hd, ad;      // plunge, pitch (counter-clockwise), rates
    double cm1, sa;           // cos(a) - 1 (computed as -2 sin^2(a/2)), sin(a)
    double pad0, pad1;
};

// Everything one instance (one mesh + body) needs on the device.  Lives in
// device memory; kernels read it through the scalar cache.
struct Inst {
    int ni, nj;
    int periodic_j;           // 1: PERIODIC2 topology, 0: O-grid or C-grid (wall + far field)
    int storage;              // 0 FP32, 1 FP16 shifted
    int tiles_i, tiles_j;     // tile grid of the fused kernel
    int tile_base;            // first work item of this instance in a batch
    int cgrid;                // C-grid: i not periodic, row 0 outside the wall is the wake cut
    int n_wake;               // C-grid: cut nodes on each side of the cut
    int wall_i0, wall_n;      // wall nodes: row 0, columns [wall_i0, wall_i0 + wall_n)
    int force_n;              // distinct wall nodes of the force polygon, from wall_i0
    int n_ff;                 // far-field nodes
    int cut_n;                // C-grid: columns whose row-1 state crosses the cut (2 (n_wake + 1))
    int pad0;
    long long n_nodes;
    double shift_ix, shift_iy, shift_jx, shift_jy;
    double dt_d;
    float gamma, Cv, Cp, mu, Pr, dt;
    float rho_inf, T_inf, ux_inf, uy_inf;
    float ref[NPOP];          // FP16 shifted storage: reference populations
    float scale[2];           // FP16 shifted storage: f, g scales
    float inv_scale[2];
    Body body;
    // device buffers (all inside the caller's workspace)
    void *pop[2];             // ping-pong [18][nj][ni], float or half
    const double2 *X;         // [nj][ni] undeformed coordinates
    uint16_t *wall_mask;      // [ni] bit k: population k missing at the wall node
    float4 *wall_tgt;         // [ni] (rho, ux, uy, T) targets
    const float2 *wall_B;     // [ni] index offsets of point B from the wall node
    const int2 *ff;           // [n_ff] far-field node index, interior node an outlet copies
    const uint8_t *inflow;    // [n_ff] far-field node is an inlet
    float *cutbuf;            // C-grid: [16][cut_n] post-collision moving populations of row 1
    double4 *wall_force;      // [ni] per-node (Fx, Fy, Mz, 0)
    const double *wall_dist;  // [nj][ni] distance to the wall (blend_mode 1), else null
    BodySlot *slots;          // [3] body states at levels n % 3
    double *history;          // [HIST_CAP][6]
    long long *step;          // completed steps
    unsigned *err;            // sticky error word
    double *scratch;          // init / dump staging (aliases the idle ping-pong side)
};

}  // namespace fsi

namespace fsi {
// host-callable launchers (fsilbm_kernels.hip)
hipError_t launch_collide_stream(const Inst *insts, const int2 *work, int n_work, int storage,
                                 hipStream_t s, int grid, bool cgrid, int shape);
hipError_t launch_cut_export(const Inst *insts, const int2 *work, int n_work, int storage,
                             hipStream_t s);
hipError_t launch_wall_targets(const Inst *insts, const int2 *work, int n_work, int storage,
                               hipStream_t s);
hipError_t launch_wall_grad_force(const Inst *insts, const int2 *work, int n_work, int storage,
                                  int phase, hipStream_t s);
hipError_t launch_body(const Inst *insts, int n_inst, int phase, hipStream_t s);
hipError_t launch_init_equilibrium(const Inst *inst, const double *macro, long long n_nodes,
                                   int storage, hipStream_t s);
hipError_t launch_dump_macro(const Inst *inst, int side, double *out, long long n_nodes, int storage,
                             hipStream_t s);
hipError_t launch_decode(const Inst *inst, int side, int q0, float *out, long long n_nodes, int storage,
                         hipStream_t s);
hipError_t launch_encode(const Inst *inst, int side, int q0, const float *in, long long n_nodes,
                         int storage, hipStream_t s);
}  // namespace fsi
