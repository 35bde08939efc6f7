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
// Tile shapes of the fused kernel, one thread per arrival node (512-thread
// workgroups, 256 for 16 x 16); the batch autotuner chooses among them.
// Instances with a cut (or two bodies) run the cut-capable build, which exists
// for shape 0 only.  A single instance without a cut whose step streams more
// than the 256 MiB Infinity Cache holds (populations read and written, and X)
// runs on WIDE_SHAPE, with non-temporal population stores: each tile row of a
// population plane is then a DRAM run of 70 consecutive nodes instead of 38;
// smaller working sets stay in the cache and keep 32 x 16.
constexpr int N_TILE_SHAPES = 4;
constexpr int TILE_SHAPES[N_TILE_SHAPES][2] = {{32, 16}, {64, 8}, {16, 32}, {16, 16}};
constexpr int WIDE_SHAPE = 1;
constexpr long long CACHE_BYTES = 256ll << 20;
// Visiting order of a single instance's tiles: N_XCD column strips, each
// strip row by row from j = 0.  The kernel gives each XCD a contiguous run of
// the list, i.e. one strip: a tile's lower neighbour follows it one strip
// width of tiles later, while the halo rows they share are still in that
// XCD's L2, and the XCDs, walking down their strips together, read whole rows
// of each population plane between them.
constexpr int N_XCD = 8;
constexpr int HIST_CAP = 1 << 16;   // force / displacement history records kept

// error bits of the device error word
constexpr unsigned ERR_CFL = 1u;    // departure point outside the node's cells
constexpr unsigned ERR_STATE = 2u;  // rho<=0, T<=0, T>=1, Phi_0<=0, NaN
constexpr unsigned ERR_MESH = 4u;   // det(dx/dxi) <= 0 after blending
// node flags of bounded Q9 meshes
constexpr uint8_t Q9_WALL = 1, Q9_FAR = 2;              // boundary nodes
constexpr uint8_t Q9_BOUNDARY = Q9_WALL | Q9_FAR;
constexpr uint8_t Q9_MOVES = 4;                         // the body's blending moves the node
constexpr uint8_t Q9_PATCH_MOVES = 8;                   // a node of its elements moves
// element flags of a moving body on a Q9 mesh
constexpr uint8_t Q9E_MOVES = 1;                        // a node of the element moves
constexpr uint8_t Q9E_RIGID = 2;                        // every node in the rigid zone

enum Dof { DOF_PRESCRIBED = 0, DOF_HEAVE = 1, DOF_PITCH_PLUNGE = 2, DOF_FIXED = 3 };

constexpr int MAX_BODIES = 2;      // bodies per instance

// Constant description of one body of an instance.
struct Body {
    int dof;
    int present;
    double m, S_a, I_a, k_h, k_a;
    double cx, cy;            // blending centre (undeformed frame)
    double ex, ey;            // rotation centre of its rigid map: its elastic axis, or
                              // the axis of the body it is linked to
    double r_rigid, inv_width;// 1 / (r_blend - r_rigid)
    double r_rigid2, r_blend2;// squared radii (r_rigid2 < 0 if r_rigid <= 0)
    double heave_amp, heave_omega, pitch_amp, pitch_omega;
    double release_time;      // > 0: prescribed motion until then (1DOF / 2DOF)
    int blend_mode;           // 0: radial from (cx, cy); 1: per-node wall distance
    int master;               // body whose equation moves it (itself unless linked)
};

// Body state at one time level, plus the rotation terms the kernels need.
struct BodySlot {
    double h, a, hd, ad;      // plunge, pitch (counter-clockwise), rates
    double cm1, sa;           // cos(a) - 1 (computed as -2 sin^2(a/2)), sin(a)
    double pad0, pad1;
};

// Everything one instance (one mesh + its bodies) needs on the device.  Lives
// in device memory; kernels read it through the scalar cache.
//
// Cut topologies (C-grid, twin O-grid): node (i, -m) is node (mirror - i, m)
// (mod ni when i is periodic).  The cut columns of row 0 are the primary
// columns cut_a < i < cut_b and their mirror images; the row-1 state of the
// columns exp_lo .. cut_b and of their mirror images crosses the cut through
// cutbuf.  Walls: n_seg column segments [seg_i0, seg_i0 + seg_n) of row 0
// (segment k belongs to body k); a segment with seg_dup = 1 ends on a second
// copy of its first point.
struct Inst {
    int ni, nj;
    int periodic_j;           // 1: PERIODIC2 topology, 0: wall + far field
    int storage;              // 0 FP32, 1 FP16 shifted
    int stream_out;           // 9-node meshes: the step streams more than the Infinity
                              // Cache holds (non-temporal population stores)
    int tiles_i, tiles_j;     // tile grid of the fused kernel
    int tile_base;            // first work item of this instance in a batch
    int cut;                  // C-grid or twin O-grid: row 0 has a cut
    int exits;                // C-grid: i not periodic, columns 0 and ni - 1 are far field
    int cut_a, cut_b, mirror; // see above
    int exp_lo;               // first exported primary column (max(cut_a, 0))
    int cut_n;                // columns whose row-1 state crosses the cut (2 (cut_b - exp_lo + 1))
    int n_seg;
    int seg_i0[MAX_BODIES], seg_n[MAX_BODIES], seg_dup[MAX_BODIES];
    int n_ff;                 // far-field nodes
    int nbody;                // bodies (0 .. MAX_BODIES)
    int n_sub;                // coupling sub-iterations per step (1: staggered)
    int pad1;
    double relax;             // sub-iteration relaxation factor
    long long n_nodes;
    double shift_ix, shift_iy, shift_jx, shift_jy;
    double dt_d;
    double gm1_d;             // gamma - 1 in FP64 (the FP64 initialisation and field output)
    float gamma, Cv, Cp, mu, Pr, dt;
    float rho_inf, T_inf, ux_inf, uy_inf;
    float ref[NPOP];          // FP16 shifted storage: reference populations
    float scale[2];           // FP16 shifted storage: f, g scales
    float inv_scale[2];
    Body body[MAX_BODIES];
    // device buffers (all inside the caller's workspace)
    void *pop[2];             // ping-pong [18][nj][ni], float or half
    const double2 *X;         // [nj][ni] undeformed coordinates
    uint16_t *wall_mask;      // [ni] bit k: population k missing at the wall node
    uint16_t *wall_amb;       // [ni] bit k: departure point within FP32 reach of the wall decision line
    float4 *wall_tgt;         // [ni] (rho, ux, uy, T) targets
    const float2 *wall_B;     // [ni] index offsets of point B from the wall node
    const int2 *ff;           // [n_ff] far-field node index, interior node an outlet copies
    const uint8_t *inflow;    // [n_ff] far-field node is an inlet
    float *cutbuf;            // cut topologies: [18][cut_n] post-collision populations of row 1 (f_1..8, g_1..8, f_0, g_0)
    double4 *wall_force;      // [ni] per-node (Fx, Fy, Mz, 0)
    const double *wall_dist;  // [nbody][nj][ni] distance to each body's wall (blend_mode 1), else null
    BodySlot *slots;          // [3][MAX_BODIES] body states at levels n % 3
    double *history;          // [MAX_BODIES][HIST_CAP][6]
    double *resid;            // [MAX_BODIES] remaining change of the last coupling sub-iteration
    long long *step;          // completed steps
    unsigned *err;            // sticky error word
    double *scratch;          // init / dump staging (aliases the idle ping-pong side)
    // unstructured 9-node meshes (topology FSI_TOPO_Q9); ni = nodes, nj = 1
    int n_elems;
    int pad2;
    const int *elems;         // [n_elems][9] node indices
    const float2 *erel;       // [n_elems][9] node positions relative to the element's centre node
    const int *patch_off;     // [n_nodes + 1] CSR offsets of each node's elements
    const int *patch_ent;     // [9 n_elems] element * 16 + the node's local index in it
    float2 *uq;               // [n_nodes] (delta Q_x, delta Q_y)
    float *us;                // [n_nodes] mu / p
    float2 *ud;               // [n_nodes] D_a = (mu / p) d_a delta Q_a
    float2 *ueg;              // [n_elems][9] element derivatives at the element's nodes
    void *upost;              // [n_nodes][8][2] post-collision moving populations (f_k, g_k), FP32,
                              // then (moving body) [n_nodes][2] the rest pair (f_0, g_0)
    int *dep_e;               // [8 or 9][n_nodes] element holding each departure point (plane 8:
                              // the rest direction of a moving body; -1 missing, -2 the node itself)
    float2 *dep_xy;           // [8 or 9][n_nodes] its local coordinates there
    // node blocks of U_BLOCK consecutive nodes for the LDS-staged interpolation
    // (null bh_off: every block gathers from device memory instead)
    int u_nblk, u_hmax, u_lemax, u_eu16;
    const int *bh_off;        // [u_nblk + 1] offsets into bh_nodes
    const int *bh_nodes;      // nodes of the elements of the block's nodes (its halo), ascending
    const int *be_off;        // [u_nblk + 1] offsets into be_elem / be_nodes
    const int *be_elem;       // elements holding a node of the block, ascending
    const uint16_t *be_nodes; // [.][u_eu16] their nine nodes as halo positions (padded)
    const uint16_t *uself;    // [n_nodes] each node's own position in its block's halo
    uint16_t *dep_le;         // [8 or 9][n_nodes] departure element as a position in the block's list
    // unstructured meshes round a fixed body: wall and far-field nodes
    int n_qw, n_qf;
    int q9_rotates;           // moving body whose rigid map may turn (else a translation)
    const uint8_t *eflag;     // [n_elems] Q9E_MOVES, Q9E_RIGID (moving body), else null
    const uint8_t *qflag;     // [n_nodes] Q9_WALL, Q9_FAR (else interior), Q9_MOVES, Q9_PATCH_MOVES
    const int *qw_nodes;      // [n_qw] wall polygon, clockwise
    const int *qw_idx;        // [n_nodes] position in qw_nodes, -1 elsewhere
    const int *qf_nodes;      // [n_qf]
    const double4 *qw_geo;    // [n_qw] (n ds)_x, (n ds)_y, x - x_ea, y - y_ea
    const int *qw_eB;         // [n_qw] element holding the point B
    const float2 *qw_xyB;     // [n_qw] local coordinates of B there
    float2 *qw_prev;          // [n_qw] (rho, T) of the completed wall node, previous level
    const int *qw_coff;       // [n_qw + 1] first patch entry of each wall node in qw_corner
    const double2 *qw_corner; // [.][4] corners of each wall node's elements relative to the node (FP64)
    // a moving body on a Q9 mesh (null: fixed)
    double2 *qdisp;           // [2][n_nodes] blended displacement at levels n, n+1
    const float2 *dgr;        // [n_nodes][3] nodal derivatives of r, r X, r Y (moving body)
    const int *patch8;        // [n_nodes][8] first patch entries (Q9 meshes), -1 past the end
};

// nodes per block of the LDS-staged interpolation
constexpr int U_BLOCK = 256;

// u16 per element in a block's element list (nine halo positions, padded):
// 16 (read as 16 + 2 bytes), 12 (8 + 8 + 2) or 10 (five 4-byte words); the
// widest whose block still lets four blocks share a CU's 160 KiB of LDS
constexpr size_t U_LDS_PER_BLOCK = 40960;

// LDS of one node block: 8 planes of (f_k, g_k) over the halo (9 with a
// moving body: the rest pair too), the element lists as halo positions, the
// block's rest populations (8-byte aligned)
__host__ __device__ inline size_t u_block_elem_bytes(int lemax, int eu16) {
    return (((size_t)lemax * eu16 * 2 + 7) / 8) * 8;
}
__host__ __device__ inline size_t u_block_lds_bytes(int hmax, int lemax, int eu16, int planes) {
    return (size_t)hmax * planes * 8 + u_block_elem_bytes(lemax, eu16) + (size_t)U_BLOCK * 8;
}

}  // namespace fsi

namespace fsi {
// host-callable launchers (fsilbm_kernels.hip)
// stream_out: the launch's step streams more than the Infinity Cache holds
// (non-temporal population stores; the wide shape only)
hipError_t launch_collide_stream(const Inst *insts, const int2 *work, int n_work, int storage,
                                 hipStream_t s, int grid, bool cut, int shape, bool stream_out = false);
hipError_t launch_cut_export(const Inst *insts, const int2 *work, int n_work, int storage,
                             hipStream_t s);
hipError_t launch_wall_targets(const Inst *insts, const int2 *work, int n_work, int storage,
                               hipStream_t s);
hipError_t launch_wall_grad_force(const Inst *insts, const int2 *work, int n_work, int storage,
                                  int phase, hipStream_t s);
hipError_t launch_body(const Inst *insts, int n_inst, int phase, hipStream_t s);
hipError_t launch_unstructured(const Inst *inst, long long n_nodes, long long n_elems, int storage,
                               float2 *uq, float2 *ud, float2 *ueg, int n_blocks, int hmax, int lemax,
                               int eu16, const double2 *disp0, int relocate, hipStream_t s);
// a moving body on a Q9 mesh: node displacements of levels n and n+1, and
// (relocate) the departure points on the moving mesh
hipError_t launch_unstructured_dep_le(const Inst *inst, long long n_nodes, hipStream_t s);
hipError_t launch_unstructured_motion(const Inst *inst, long long n_nodes, long long n_elems, int relocate,
                                      hipStream_t s);
hipError_t launch_unstructured_locate(const Inst *inst, long long n_nodes, hipStream_t s);
hipError_t launch_unstructured_moments(const Inst *inst, long long n_nodes, int storage, hipStream_t s);
// far field, wall targets, Grad populations and traction (phase 1), or
// traction and wall values of the current level only (phase 0)
hipError_t launch_unstructured_boundary(const Inst *inst, int n_wall, int n_far, int storage, int phase,
                                        hipStream_t s);
hipError_t launch_init_equilibrium(const Inst *inst, const double *macro, long long n_nodes,
                                   int storage, hipStream_t s);
hipError_t launch_dump_macro(const Inst *inst, int side, double *out, long long n_nodes, int storage,
                             hipStream_t s);
hipError_t launch_decode(const Inst *inst, int side, int q0, float *out, long long n_nodes, int storage,
                         hipStream_t s);
hipError_t launch_encode(const Inst *inst, int side, int q0, const float *in, long long n_nodes,
                         int storage, hipStream_t s);
}  // namespace fsi
