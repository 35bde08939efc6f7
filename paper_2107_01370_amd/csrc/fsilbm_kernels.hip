// gfx950 kernels of the two-population compressible lattice Boltzmann FSI step
// (Bhadauria, Dorschner & Karlin, arXiv 2107.01370).
//
//   k_collide_stream   fused collision (Sec. II.C) + ALE semi-Lagrangian
//                      streaming (Sec. II.A-B) over 32 x 16 node tiles
//   k_cut_export       C-grid pre-pass: row-1 post-collision state of the cut
//   k_wall_targets     Grad targets at the wall (Sec. III.A.1) and
//                      far-field equilibria (Sec. III.A.2)
//   k_wall_grad_force  Grad populations at the wall and per-node traction
//                      (Sec. III.A.1, Sec. III force)
//   k_body             deterministic force reduction + rigid-body RK4 (Sec. IV)
//   k_init_equilibrium, k_dump_macro, k_decode, k_encode: set-up and I/O
// (the unstructured 9-node element path is in fsilbm_unstructured.hip; the
// collision and the population accessors both use are in fsilbm_device.h)
//
// Precision: populations are stored in FP32 (or FP16 as shifted deviations)
// and collided / interpolated in FP32.  Mesh coordinates, blending weights,
// mesh displacements, the traction sum and the body ODE are FP64; coordinate
// differences are formed in FP64 and only then rounded to FP32.
#include "fsilbm_device.h"
#include "fsilbm_wall.h"

namespace fsi {

// ---------------------------------------------------------------------------
// Fused collision + ALE interpolating streaming.
//
// One workgroup of TX * TY threads owns a TX x TY block of arrival nodes
// (32 x 16 by default; 64 x 8, 16 x 32 and 16 x 16 are the other shapes the
// batch autotuner tries).  The momentum
// correction needs nested gradients (reach 2) and the interpolation stencil
// reaches one node, so the tile is processed with a halo of 3:
//   phase 1 (tile+3): populations -> delta Q_a, mu/p;  mesh geometry -> LDS
//   phase 2 (tile+2): D_a = (mu/p) d_{x_a} dQ_a on the mesh x^n     -> LDS
//   phase 3 (tile+1): F_a = d_{x_a} D_a; collide                     -> LDS
//   phase 4 (tile)  : departure points on x^{n+1}, 3x3 Lagrange
//                     interpolation from LDS, store f^{n+1}, g^{n+1}
//
// Geometry in LDS, all FP32 and relative to FP64 references of the tile (its
// centre node's undeformed position and blended displacement at t^n): the
// undeformed coordinates X - X_ref (with periodic shifts), the displacement at
// t^n minus D_ref (dn) and the increment over the step (dd), each formed in
// FP64 and rounded once.  Coordinate differences inside a tile are then single
// FP32 subtractions whose rounding is ~1e-7 of the tile's extent (a few 1e-6
// of a cell), on meshes with large absolute coordinates and displacements;
// integer grids stay exact.
// ---------------------------------------------------------------------------
constexpr int NMOV = 16;     // moving populations in the row-1 export (f_1..8, g_1..8) ...
constexpr int NFG = NMOV + 2; // ... and the rest pair (f_0, g_0)
// waves per SIMD the launch bounds ask for (16 waves per CU: two 512-thread or
// four 256-thread workgroups), which caps the VGPRs at 128
constexpr int kWavesPerSimd = 4;

// extents of the tile and its halo rings for a TX x TY tile
template <int TX, int TY>
struct Geo {
    static constexpr int TILE_X = TX, TILE_Y = TY;
    static constexpr int NT = TX * TY;                 // threads: one arrival node each
    static constexpr int R3X = TX + 6, R3Y = TY + 6, R3N = R3X * R3Y;
    static constexpr int R2X = TX + 4, R2Y = TY + 4, R2N = R2X * R2Y;
    static constexpr int R1X = TX + 2, R1Y = TY + 2, R1N = R1X * R1Y;
    static constexpr int RING_ROWS = 2 * 2 * R3X;     // two rows above and below R1
    static constexpr int R1_ROUNDS = (R1N + NT - 1) / NT;
    static_assert(R1_ROUNDS == 2, "phase-1/3 register hand-off assumes two rounds");
    static_assert(R3N <= 2 * NT && R2N <= 2 * NT, "two rounds per phase");
};

template <class G>
struct K1Smem {
    float2 Xu[G::R3N];       // X - X_ref (undeformed, periodic shifts applied)
    float2 dn[G::R3N];       // (1 - r) d^n(X) - D_ref^n
    float2 dd[G::R3N];       // (1 - r)(d^{n+1}(X) - d^n(X))
    float2 D[G::R2N];        // nested correction, first level
    union {
        struct {
            float Qx[G::R3N], Qy[G::R3N], S[G::R3N];
        } q;
        // post-collision pairs (f_k, g_k), k = 0..8, of each tile+1 node (the
        // rest pair only on a tile whose mesh moves), node-major: one 8-byte
        // read per stencil tap serves both populations, and the three taps of
        // a stencil row, for all nine directions, lie within the reach of one
        // base address (consecutive lanes 72 bytes apart: no bank conflicts)
        float2 FG[G::R1N][9];
    } u;
};

// index-space first derivative: centred, or one-sided 3-point on a wall row,
// the far-field row and the exit columns of a C-grid
struct Sten {
    int o1, o2;              // offsets (in nodes along the index) of the two other nodes
    float w1, w2;            // d = w1 (C_o1 - C_0) + w2 (C_o2 - C_0) ...
    bool centred;            // ... or (C_{+1} - C_{-1}) / 2
};

__device__ __forceinline__ Sten centred_sten() {
    Sten s;
    s.centred = true; s.o1 = 1; s.o2 = -1; s.w1 = 0.5f; s.w2 = -0.5f;
    return s;
}

__device__ __forceinline__ Sten forward_sten(int dir) {
    Sten s;
    s.centred = false; s.o1 = dir; s.o2 = 2 * dir; s.w1 = 2.0f * (float)dir; s.w2 = -0.5f * (float)dir;
    return s;
}

// a cx + b cy + c for lattice velocity components cx, cy in {-1, 0, 1} (known
// once a loop over the directions is unrolled: no products, no terms for 0)
__device__ __forceinline__ float affine(int cx, int cy, float a, float b, float c) {
    float r = c;
    if (cx != 0) r = cx > 0 ? r + a : r - a;
    if (cy != 0) r = cy > 0 ? r + b : r - b;
    return r;
}

// column across the cut from column i (cut topologies)
__device__ __forceinline__ int mirror_col(const Inst &P, int i) {
    const int m = P.mirror - i;
    return P.exits ? m : wrap(m, P.ni);
}

// cut column of row 0: a primary cut column or the mirror image of one
__device__ __forceinline__ bool cut_col(const Inst &P, int i) {
    const int m = mirror_col(P, i);
    return (i > P.cut_a && i < P.cut_b) || (m > P.cut_a && m < P.cut_b);
}

// wall column: the whole row 0 of an O-grid, every column of row 0 but the
// cut ones on a cut topology.  `cg` (cut topology) is a compile-time false in
// the kernels built without cut support, which folds every cut branch away.
__device__ __forceinline__ bool wall_col(const Inst &P, int ig, bool cg) {
    return !cg || !cut_col(P, wrap(ig, P.ni));
}
__device__ __forceinline__ bool wall_col(const Inst &P, int ig) { return wall_col(P, ig, P.cut); }

// a copy of a duplicated wall point (C-grid trailing edge, twin junction)
__device__ __forceinline__ bool dup_point(const Inst &P, int i) {
    for (int k = 0; k < P.n_seg; ++k)
        if (P.seg_dup[k] && (i == P.seg_i0[k] || i == P.seg_i0[k] + P.seg_n[k] - 1)) return true;
    return false;
}

// along j at (unwrapped) node (ig, jg); rows below 0 of a cut topology are
// across the cut
__device__ __forceinline__ Sten jstencil(const Inst &P, int ig, int jg, bool cg) {
    if (!P.periodic_j) {
        if (jg == P.nj - 1) return forward_sten(-1);
        if (jg == 0 && wall_col(P, ig, cg)) return forward_sten(1);
    }
    return centred_sten();
}

__device__ __forceinline__ Sten istencil(const Inst &P, int ig, bool cg) {
    if (cg && P.exits) {
        if (ig == 0) return forward_sten(1);
        if (ig == P.ni - 1) return forward_sten(-1);
    }
    return centred_sten();
}

// derivative of an LDS field at entry c with `stride` entries per index step
__device__ __forceinline__ float dsten(const float *F, int c, int stride, const Sten &s) {
    if (s.centred) return 0.5f * (F[c + stride] - F[c - stride]);
    const float f0 = F[c];
    return s.w1 * (F[c + s.o1 * stride] - f0) + s.w2 * (F[c + s.o2 * stride] - f0);
}

// does local (unwrapped) node (ig, jg) exist: periodic indices always, rows
// below 0 of a cut topology through the mirror across the cut
__device__ __forceinline__ bool node_exists(const Inst &P, int ig, int jg, bool cg) {
    if (P.periodic_j) return true;
    if (cg) return (!P.exits || (ig >= 0 && ig < P.ni)) && jg < P.nj;
    return jg >= 0 && jg < P.nj;
}

// cut topologies: slot of column i (in [0, ni)) in the row-1 export buffer
// (-1: not exported): the primary columns exp_lo .. cut_b, then their mirrors
__device__ __forceinline__ int cut_slot(const Inst &P, int i) {
    const int half = P.cut_b - P.exp_lo + 1;
    if (i >= P.exp_lo && i <= P.cut_b) return i - P.exp_lo;
    const int m = mirror_col(P, i);
    if (m >= P.exp_lo && m <= P.cut_b) return half + (m - P.exp_lo);
    return -1;
}

// position difference x_a - x_b of two R3 entries; `level1` adds the step
// increment (mesh at t^{n+1})
template <class G>
__device__ __forceinline__ float2 pos_diff(const K1Smem<G> &sm, int a, int b, bool level1) {
    float2 d;
    d.x = (sm.Xu[a].x - sm.Xu[b].x) + (sm.dn[a].x - sm.dn[b].x);
    d.y = (sm.Xu[a].y - sm.Xu[b].y) + (sm.dn[a].y - sm.dn[b].y);
    if (level1) {
        d.x += sm.dd[a].x - sm.dd[b].x;
        d.y += sm.dd[a].y - sm.dd[b].y;
    }
    return d;
}

// lane mask of a per-lane condition over the active lanes, and a lane's bit of
// a wave-uniform mask (selects on such bits take the mask as their condition)
__device__ __forceinline__ uint64_t ballot(bool c) { return __builtin_amdgcn_ballot_w64(c); }
__device__ __forceinline__ bool lane_bit(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// rigid-map terms of ring level l (0, 1 or 2; wave-uniform) as a body slot
__device__ __forceinline__ BodySlot level_slot(int l, double h0, double c0, double s0, double h1,
                                               double c1, double s1, double h2, double c2,
                                               double s2) {
    BodySlot b;
    b.h = l == 0 ? h0 : (l == 1 ? h1 : h2);
    b.cm1 = l == 0 ? c0 : (l == 1 ? c1 : c2);
    b.sa = l == 0 ? s0 : (l == 1 ? s1 : s2);
    b.a = 0.0; b.hd = 0.0; b.ad = 0.0; b.pad0 = 0.0; b.pad1 = 0.0;
    return b;
}

// an opaque register copy: the value is computed where it is defined and
// kept, not re-derived from its inputs at each later use
__device__ __forceinline__ void keep(float &x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void keep(float3 &v) { keep(v.x); keep(v.y); keep(v.z); }

// undeformed position of R3 entry a relative to Xc
template <class G>
__device__ __forceinline__ float2 rel_pos(const K1Smem<G> &sm, int a, float2 Xc) {
    return make_float2(sm.Xu[a].x - Xc.x, sm.Xu[a].y - Xc.y);
}

// coefficients (of c_x, of c_y, constant) of E x P for a target P = M c + P0
__device__ __forceinline__ float3 side_coef(float2 E, float m11, float m12, float m21, float m22,
                                            float P0x, float P0y) {
    return make_float3(E.x * m21 - E.y * m11, E.x * m22 - E.y * m12, E.x * P0y - E.y * P0x);
}

// inverse data of a bilinear cell X(u, v) = u e_i + v e_j + u v tw spanned from
// the node by the edges e_i, e_j with far corner K: 1/(e_i x e_j) and the twist
// coefficients tu = (tw x e_j)/(e_i x e_j), tv = (e_i x tw)/(e_i x e_j)
struct CellInv {
    float im, tu, tv;
};

__device__ __forceinline__ CellInv cell_inv(float2 ei, float2 ej, float2 K) {
    const float twx = K.x - ei.x - ej.x, twy = K.y - ei.y - ej.y;
    CellInv c;
    c.im = rcpf(ei.x * ej.y - ei.y * ej.x);
    c.tu = c.im * (twx * ej.y - twy * ej.x);
    c.tv = c.im * (ei.x * twy - ei.y * twx);
    return c;
}

// metric (x_xi, x_eta, y_xi, y_eta) at R3 entry c
template <class G>
__device__ __forceinline__ void metric(const K1Smem<G> &sm, int c, const Sten &is, const Sten &js,
                                       bool level1, float J[4]) {
    constexpr int R3X = G::R3X;
    if (is.centred) {
        const float2 di = pos_diff(sm, c + 1, c - 1, level1);
        J[0] = 0.5f * di.x;
        J[2] = 0.5f * di.y;
    } else {
        const float2 d1 = pos_diff(sm, c + is.o1, c, level1);
        const float2 d2 = pos_diff(sm, c + is.o2, c, level1);
        J[0] = is.w1 * d1.x + is.w2 * d2.x;
        J[2] = is.w1 * d1.y + is.w2 * d2.y;
    }
    if (js.centred) {
        const float2 dj = pos_diff(sm, c + R3X, c - R3X, level1);
        J[1] = 0.5f * dj.x;
        J[3] = 0.5f * dj.y;
    } else {
        const float2 d1 = pos_diff(sm, c + js.o1 * R3X, c, level1);
        const float2 d2 = pos_diff(sm, c + js.o2 * R3X, c, level1);
        J[1] = js.w1 * d1.x + js.w2 * d2.x;
        J[3] = js.w1 * d1.y + js.w2 * d2.y;
    }
}

// Undeformed neighbourhood, mesh metric at t^{n+1} and mesh velocity of one
// arrival node, gathered by the caller from its LDS layout.
struct NodeGeo {
    float J[4];                       // dx^{n+1}/dxi: x_xi, x_eta, y_xi, y_eta
    float2 Epi, Emi, Epj, Emj;        // X of the neighbours +i, -i, +j, -j minus X
    float2 Kpp, Kmp, Kmm, Kpm;        // far corners of the cells (+i+j, -i+j, -i-j, +i-j)
    float2 E2;                        // X two rows up minus X (wall row only)
    float VGx, VGy;                   // V_G = (x^{n+1} - x^n)/dt
};

// ALE semi-Lagrangian streaming of one arrival node (Sec. II.A-B): for each
// population (the rest pair only if `rest`), the departure point
// X - dt g^{-1}(c_i - V_G), its cell and local coordinates in the undeformed
// mesh (bilinear element), and the 9-node quadratic Lagrange interpolation of
// the post-collision pairs FG (node-major, FGX nodes per row; cn: the node's own
// entry).  Stores the new populations at byte offset `off` or, DEFER, leaves
// them in out[] (f_0..8, g_0..8) for the caller to store; on a wall node the
// missing (miss) and near-line (amb) populations are flagged instead.
template <int STORE, int FGX, bool DEFER = false, bool NT = false>
__device__ __forceinline__ void node_stream(const Inst &P, const PopBuf &dst, int off,
                                            const NodeGeo &ng, bool wall, bool rest,
                                            const float2 (*FG)[9], int cn, float dtf,
                                            uint16_t &miss, uint16_t &amb, unsigned &err,
                                            float *out = nullptr) {
    const float2 Epi = ng.Epi, Emi = ng.Emi, Epj = ng.Epj, Emj = ng.Emj;
    // centred metric of X (one-sided into the fluid on the wall row)
    const float BXxi = 0.5f * (Epi.x - Emi.x), BYxi = 0.5f * (Epi.y - Emi.y);
    float BXeta, BYeta;
    if (wall) {
        BXeta = 2.0f * Epj.x - 0.5f * ng.E2.x;
        BYeta = 2.0f * Epj.y - 0.5f * ng.E2.y;
    } else {
        BXeta = 0.5f * (Epj.x - Emj.x);
        BYeta = 0.5f * (Epj.y - Emj.y);
    }
    const float VGx = ng.VGx, VGy = ng.VGy;
    const float *J = ng.J;
    const float det = J[0] * J[3] - J[2] * J[1];
    if (!(det > 0.0f)) err |= ERR_MESH;
    const float idet = rcpf(det);
    // linear departure offsets are affine in c_i:
    //   dxi_i = -dt (dx^{n+1}/dxi)^{-1} (c_i - V_G) = A c_i + B0,
    // and so is the target X_dp - X = (dX/dxi) dxi_i = (B A) c_i + B B0
    const float a11 = -dtf * idet * J[3], a12 = dtf * idet * J[1];
    const float a21 = dtf * idet * J[2], a22 = -dtf * idet * J[0];
    const float B0x = -(a11 * VGx + a12 * VGy), B0y = -(a21 * VGx + a22 * VGy);
    const float p11 = BXxi * a11 + BXeta * a21, p12 = BXxi * a12 + BXeta * a22;
    const float p21 = BYxi * a11 + BYeta * a21, p22 = BYxi * a12 + BYeta * a22;
    const float P0x = BXxi * B0x + BXeta * B0y, P0y = BYxi * B0x + BYeta * B0y;
    // Side of each edge E on which the target lies: E x (X_dp - X), also
    // affine in c_i (the same coefficients serve all nine directions)
    float3 Spi = side_coef(Epi, p11, p12, p21, p22, P0x, P0y);
    float3 Smi = side_coef(Emi, p11, p12, p21, p22, P0x, P0y);
    float3 Spj = side_coef(Epj, p11, p12, p21, p22, P0x, P0y);
    float3 Smj = side_coef(Emj, p11, p12, p21, p22, P0x, P0y);
    // formed once here for all directions (not re-derived per direction)
    keep(Spi); keep(Smi); keep(Spj); keep(Smj);
    // the four cells round the node as first-order (bilinear) elements
    // X(u, v) = u e_i + v e_j + u v tw, (u, v) in [0,1]^2, with e_i, e_j
    // the edges along which the cell extends: 1/(e_i x e_j) and the twist
    // terms of the inverse map, once per node.  Cell (li, lj) extends to
    // -i if li and to -j if lj (on the wall row only cells above exist:
    // the lower pair is formed from placeholder entries and never chosen).
    const CellInv q00 = cell_inv(Epi, Epj, ng.Kpp);
    const CellInv q10 = cell_inv(Emi, Epj, ng.Kmp);
    const CellInv q11 = cell_inv(Emi, Emj, ng.Kmm);
    const CellInv q01 = cell_inv(Epi, Emj, ng.Kpm);
    const int vc = wall ? 1 : 0;                   // stencil centre row offset
    const int c1 = cn + vc * FGX;                  // stencil centre
    float cfl = 0.0f;          // largest |index offset| of the departure points
    bool unsettled = false;    // a bilinear solve that did not settle
    // the wave holds a wall node (wave-uniform): the wall decision below
    const uint64_t wall_m = ballot(wall);
    const bool wall_wave = wall_m != 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if (k == 0 && !rest) continue;           // the caller stores it
        const int cx = CXK(k), cy = CYK(k);
        const float spi = affine(cx, cy, Spi.x, Spi.y, Spi.z);
        const float smi = affine(cx, cy, Smi.x, Smi.y, Smi.z);
        const float spj = affine(cx, cy, Spj.x, Spj.y, Spj.z);
        const float smj = affine(cx, cy, Smj.x, Smj.y, Smj.z);
        // The edges split the plane round the node into four sectors, one
        // per cell; the target lies counter-clockwise of the sector's first
        // edge and clockwise of its second: (+i, +j) cell 00, (+j, -i) 10,
        // (-i, -j) 11, (-j, +i) 01.  On the wall row the cell above on the
        // target's side of the +j edge is taken (a point below the wall
        // line then has v < 0).
        // (the sector logic on the wave's lane masks: scalar instructions)
        const uint64_t sa = ballot(spi > 0.0f), sb = ballot(spj > 0.0f);
        const uint64_t sc = ballot(smi > 0.0f), sd = ballot(smj > 0.0f);
        const uint64_t s3 = sc & ~sd;
        const bool li = lane_bit((wall_m & sb) | (~wall_m & ((sb & ~sc) | s3)));
        const bool lj = lane_bit(~wall_m & (s3 | (sd & ~sa)));
        // bilinear inverse in that cell: u + tu u v = pu, v + tv u v = pv
        // with pu = (X_dp - X) x e_j / (e_i x e_j), pv = e_i x (X_dp - X) / (e_i x e_j)
        const CellInv cq = lj ? (li ? q11 : q01) : (li ? q10 : q00);
        const float pu = -cq.im * (lj ? smj : spj);
        const float pv = cq.im * (li ? smi : spi);
        const float tu = cq.tu, tv = cq.tv;
        // Fixed point from the linear solution, until an update falls below
        // 1e-6 of a cell.  Each round multiplies the error by about
        // |t| |(u, v)|, the twist relative to the cell (1e-3 on smooth
        // meshes, where the second round's update is already below the
        // bound and leaves an error at FP32 round-off): one round, a second
        // whose update is checked, and where it still moved the point
        // (strongly distorted cells; NaN never settles) up to 20 in all
        float uu, vv;
        {
            const float uv = pu * pv;
            uu = pu - tu * uv;
            vv = pv - tv * uv;
        }
        {
            const float uv = uu * vv;
            const float nu = pu - tu * uv, nv = pv - tv * uv;
            bool moving = !(fabsf(nu - uu) + fabsf(nv - vv) <= 1e-6f);
            uu = nu;
            vv = nv;
            if (__any(moving)) {
#pragma unroll 1
                for (int it = 2; it < 20 && __any(moving); ++it) {
                    const float uv2 = uu * vv;
                    const float nu2 = pu - tu * uv2, nv2 = pv - tv * uv2;
                    moving = !(fabsf(nu2 - uu) + fabsf(nv2 - vv) <= 1e-6f);
                    uu = nu2;
                    vv = nv2;
                }
                unsettled = unsettled || moving;
            }
        }
        const float a = li ? -uu : uu;
        float bb = lj ? -vv : vv;
        if (wall_wave) {
            // a point more than 1e-4 of the cell below the wall line lies
            // in the body (nearer, it counts as on the line).  Within 1e-5
            // of that line (several times the FP32 error of vv) the
            // population is interpolated here and the wall kernel decides
            // in FP64.
            const bool near = wall && vv < -0.9e-4f;
            amb |= near ? (uint16_t)(1u << k) : (uint16_t)0;
            if (wall && vv < -1.1e-4f) {
                miss |= (uint16_t)(1u << k);
                continue;
            }
        }
        cfl = fmaxf(cfl, fmaxf(fabsf(a), fabsf(bb)));
        bb -= (float)vc;
        // weights of the nodes -1 and +1: a (a - 1) / 2 and a (a + 1) / 2
        const float ha = 0.5f * a, hb = 0.5f * bb;
        const float wam = fmaf(ha, a, -ha), wap = wam + a;
        const float wbm = fmaf(hb, bb, -hb), wbp = wbm + bb;
        // tensor-product quadratic Lagrange, as centre + weighted differences
        // so that constants are reproduced exactly
        float2 row[3];
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
            const float2 *F = FG[c1 + dj * FGX - 1] + k;
            const float2 fm = F[0], fc = F[9], fp = F[18];
            row[dj + 1].x = fc.x + wam * (fm.x - fc.x) + wap * (fp.x - fc.x);
            row[dj + 1].y = fc.y + wam * (fm.y - fc.y) + wap * (fp.y - fc.y);
        }
        const float outf = row[1].x + wbm * (row[0].x - row[1].x) + wbp * (row[2].x - row[1].x);
        const float outg = row[1].y + wbm * (row[0].y - row[1].y) + wbp * (row[2].y - row[1].y);
        if constexpr (DEFER) {
            out[k] = outf;
            out[Q + k] = outg;
        } else {
            pop_st<STORE, NT>(P, dst, k, off, outf);
            pop_st<STORE, NT>(P, dst, Q + k, off, outg);
        }
    }
    // a departure point beyond the node's cells (NaN sets `unsettled`), or
    // a bilinear solve that did not settle in 20 rounds
    // a departure point beyond the node's cells (NaN sets `unsettled`), or
    // a bilinear solve that did not settle in 20 rounds
    if (!(cfl <= 1.0f + 1e-4f) || unsettled) err |= ERR_CFL;
}

// Phase-1 work item p -> R3 entry: the tile+1 region first (row-major), then
// the ring of tile+3 outside it, so that a thread's phase-1 items below R1N
// are exactly its phase-3 collision nodes (their populations stay in
// registers between the two phases).
template <class G>
__device__ __forceinline__ int phase1_entry(int p) {
    constexpr int R1N = G::R1N, R1X = G::R1X, R3X = G::R3X, R3Y = G::R3Y, RING_ROWS = G::RING_ROWS;
    if (p < R1N) return (p / R1X + 2) * R3X + (p % R1X + 2);
    const int q = p - R1N;
    if (q < RING_ROWS) {
        const int r = q / R3X, c = q % R3X;
        const int row = r < 2 ? r : R3Y - 4 + r;   // rows 0, 1, R3Y-2, R3Y-1
        return row * R3X + c;
    }
    const int q2 = q - RING_ROWS;                 // columns 0, 1, R3X-2, R3X-1 of rows 2..R3Y-3
    const int row = 2 + q2 / 4, k = q2 % 4;
    const int col = k < 2 ? k : R3X - 4 + k;
    return row * R3X + col;
}

// one work item (instance, tile) of the fused kernel.  EXPORT: the C-grid
// pre-pass, which stops after the collision and writes the row-1 post-collision
// populations of the cut columns to P.cutbuf (the tiles across the cut read
// them as their row -1 instead of colliding there: a node below the cut seen
// from the other side has different neighbours on row 0 next to the trailing
// edge, so its collision cannot be formed in the mirrored frame).
template <int STORE, bool EXPORT, bool CG, int TX, int TY, bool NT = false>
__device__ __forceinline__ void collide_stream_tile(K1Smem<Geo<TX, TY>> &sm,
                                                    const Inst *__restrict__ insts, const int2 item) {
    using G = Geo<TX, TY>;
    constexpr int TILE_X = TX, TILE_Y = TY;
    constexpr int R3X = G::R3X, R3N = G::R3N, R2X = G::R2X, R2N = G::R2N;
    constexpr int R1X = G::R1X, R1N = G::R1N, R1_ROUNDS = G::R1_ROUNDS;
    constexpr int K1_THREADS = G::NT;
    const Inst &P = insts[item.x];
    const bool cg = CG && P.cut;
    // bodies whose regions the tile may see (one in the kernels built
    // without cut support, which serve meshes with at most one body)
    constexpr int NB = CG ? MAX_BODIES : 1;
    const int tile = item.y;
    const int tiles_i = (P.ni + TX - 1) / TX;
    const int ti = tile % tiles_i, tj = tile / tiles_i;
    const int i0 = ti * TILE_X, j0 = tj * TILE_Y;
    const int ni = P.ni, nj = P.nj;
    const int t = threadIdx.x;
    unsigned err = 0;
    // The tile's state of the step, requested in one round: the step counter,
    // the body states of all three ring levels (the pair the step needs is
    // picked once the counter is in), both population buffers and the FP64
    // reference node (all written by earlier kernels only, so read through
    // the scalar cache)
    // (the tile's centre node: the largest coordinate relative to it, and so
    // the FP32 rounding of the LDS geometry, is half that from a corner)
    const long long iref = (long long)min(j0 + TY / 2, nj - 1) * ni + min(i0 + TX / 2, ni - 1);
    const long long *const stepp = P.step;
    const BodySlot *const slots = P.slots;
    const double2 *const Xp = P.X;
    void *const pop0 = P.pop[0], *const pop1 = P.pop[1];
    const long long nraw = sload(stepp);
    // rigid-map terms (h, cos a - 1, sin a) of every body at the three levels
    double rh[3][NB], rc[3][NB], rs[3][NB];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const BodySlot *sl = slots + l * MAX_BODIES + k;
            rh[l][k] = sload(&sl->h);
            rc[l][k] = sload(&sl->cm1);
            rs[l][k] = sload(&sl->sa);
        }
    const double2 Xref = sload(Xp + iref);
    const Body *const bd = P.body;
    const long long n = uniform(nraw);
    const int l0 = (int)(n % 3), l1 = l0 == 2 ? 0 : l0 + 1;
    BodySlot sn[NB], sn1[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        sn[k] = level_slot(l0, rh[0][k], rc[0][k], rs[0][k], rh[1][k], rc[1][k], rs[1][k],
                           rh[2][k], rc[2][k], rs[2][k]);
        sn1[k] = level_slot(l1, rh[0][k], rc[0][k], rs[0][k], rh[1][k], rc[1][k], rs[1][k],
                            rh[2][k], rc[2][k], rs[2][k]);
    }
    const PopBuf src = pop_buf<STORE>(P, (n & 1) ? pop1 : pop0);
    const PopBuf dst = pop_buf<STORE>(P, (n & 1) ? pop0 : pop1);
    const int nbody = min(P.nbody, NB);

    // FP64 references of the tile: position and displacement of its centre node
    const double Xrx = Xref.x, Xry = Xref.y;
    double Drx = 0.0, Dry = 0.0;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        if (k >= nbody || !bd[k].present) continue;
        const double r = uniform(blend_factor(P, k, iref, Xrx, Xry));
        double dx, dy;
        rigid_disp(bd[k], sn[k], Xrx, Xry, dx, dy);
        Drx += (1.0 - r) * dx;
        Dry += (1.0 - r) * dy;
    }

    // populations of this thread's collision nodes, kept from phase 1
    float fk[R1_ROUNDS][9], gk[R1_ROUNDS][9];
    int mv = 0;              // a node of this thread's phase-1 items moves

    // ---- phase 1: tile+3 --------------------------------------------------
    // This thread's items (two rounds): entries, node indices and periodic
    // shifts first, then every load of both items in flight together (a
    // missing item's loads fall outside their buffers: no traffic, zeros)
    constexpr int P1 = (R3N + K1_THREADS - 1) / K1_THREADS;
    static_assert(P1 == R1_ROUNDS, "phase-1 rounds hand populations to phase 3");
    int p1e[P1], p1idx[P1], p1wi[P1], p1wj[P1];
    bool p1ok[P1];
#pragma unroll
    for (int rd = 0; rd < P1; ++rd) {
        const int p = rd * K1_THREADS + t;
        const int e = phase1_entry<G>(min(p, R3N - 1));
        const int u = e % R3X, v = e / R3X;
        int ig = i0 - 3 + u, jg = j0 - 3 + v;
        // wrap into the mesh; a node seen across a periodic seam has its
        // coordinates shifted by the period; on a cut topology node (i, -m) is
        // node (mirror - i, m) across the cut (no shifts on these meshes)
        int wi = 0, wj = 0;
        bool valid = p < R3N;
        if (cg) {
            if (jg < 0) { ig = P.mirror - ig; jg = -jg; }
            if (P.exits) {
                valid = valid && ig >= 0 && ig < ni && jg < nj;
            } else {
                ig = wrap(ig, ni);
                valid = valid && jg < nj;
            }
        } else {
            if (ig < 0 || ig >= ni) {        // meshes narrower than the halo wrap more than once
                while (ig < 0) { ig += ni; --wi; }
                while (ig >= ni) { ig -= ni; ++wi; }
            }
            if (P.periodic_j) {
                if (jg < 0 || jg >= nj) {
                    while (jg < 0) { jg += nj; --wj; }
                    while (jg >= nj) { jg -= nj; ++wj; }
                }
            } else {
                valid = valid && (jg >= 0 && jg < nj);
            }
        }
        p1e[rd] = e;
        p1idx[rd] = valid ? jg * ni + ig : 0;
        p1wi[rd] = wi;
        p1wj[rd] = wj;
        p1ok[rd] = valid;
    }
    const XBuf xb = x_buf(P);
    unsigned raw[P1][NPOP];
    double2 Xr[P1];
#pragma unroll
    for (int rd = 0; rd < P1; ++rd) {
        const int off = p1ok[rd] ? pop_off<STORE>(p1idx[rd]) : kOutside;
#pragma unroll
        for (int q = 0; q < NPOP; ++q) raw[rd][q] = pop_ld_raw<STORE>(src, q, off);
        Xr[rd] = x_ld(xb, p1ok[rd] ? p1idx[rd] * 16 : kOutside);
    }
#pragma unroll
    for (int rd = 0; rd < P1; ++rd) {
        const int p = rd * K1_THREADS + t;
        if (p >= R3N) break;
        const int e = p1e[rd];
        if (!p1ok[rd]) {
            sm.Xu[e] = make_float2(0.0f, 0.0f);
            sm.dn[e] = make_float2(0.0f, 0.0f); sm.dd[e] = make_float2(0.0f, 0.0f);
            sm.u.q.Qx[e] = 0.0f; sm.u.q.Qy[e] = 0.0f; sm.u.q.S[e] = 0.0f;
            continue;
        }
        const int idx = p1idx[rd];
        // blending factors and displacements from the unshifted node: every
        // body moves the nodes of its own region of influence
        double a0x = 0.0, a0y = 0.0, a1x = 0.0, a1y = 0.0;
        bool moved = false;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            if (k >= nbody || !bd[k].present) continue;
            const double r = blend_factor(P, k, idx, Xr[rd].x, Xr[rd].y);
            if (r < 1.0) {
                double d0x, d0y, d1x, d1y;
                rigid_disp(bd[k], sn[k], Xr[rd].x, Xr[rd].y, d0x, d0y);
                rigid_disp(bd[k], sn1[k], Xr[rd].x, Xr[rd].y, d1x, d1y);
                const double om = 1.0 - r;
                a0x += om * d0x;
                a0y += om * d0y;
                a1x += om * (d1x - d0x);
                a1y += om * (d1y - d0y);
                moved = true;
            }
        }
        float2 dn = make_float2((float)(-Drx), (float)(-Dry)), dd = make_float2(0.0f, 0.0f);
        mv |= moved ? 1 : 0;
        if (moved) {
            dn = make_float2((float)(a0x - Drx), (float)(a0y - Dry));
            dd = make_float2((float)a1x, (float)a1y);
        }
        double sx = Xr[rd].x - Xrx, sy = Xr[rd].y - Xry;
        const int wi = p1wi[rd], wj = p1wj[rd];
        if (wi | wj) {            // seen across a periodic seam
            sx += (double)wi * P.shift_ix + (double)wj * P.shift_jx;
            sy += (double)wi * P.shift_iy + (double)wj * P.shift_jy;
        }
        sm.Xu[e] = make_float2((float)sx, (float)sy);
        sm.dn[e] = dn;
        sm.dd[e] = dd;
        float f[9], g[9];
        float sf = 0.0f, sg = 0.0f;            // FP16 scales of f and g, in vector registers
        if constexpr (STORE != 0) {
            sf = P.scale[0];
            sg = P.scale[1];
            keep(sf);
            keep(sg);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            f[k] = pop_decode<STORE>(P, k, raw[rd][k], sf);
            g[k] = pop_decode<STORE>(P, Q + k, raw[rd][Q + k], sg);
        }
        if (rd < R1_ROUNDS && p < R1N) {
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                fk[rd][k] = f[k];
                gk[rd][k] = g[k];
            }
        }
        const float rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
        const float jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
        const float jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
        const float G = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
        const float ir = rcpf(rho);
        const float ux = jx * ir, uy = jy * ir;
        const float T = (0.5f * G * ir - 0.5f * (ux * ux + uy * uy)) * (P.gamma - 1.0f);
        const float one3T = 1.0f - 3.0f * T;
        // delta Q_a = rho u_a (1 - 3T) - rho u_a^3
        sm.u.q.Qx[e] = jx * (one3T - ux * ux);
        sm.u.q.Qy[e] = jy * (one3T - uy * uy);
        sm.u.q.S[e] = P.mu * rcpf(rho * T);       // (1/omega - 1/2) dt = mu / p
    }
    // Rest populations (c_0 = 0) have the transformed velocity -g^{-1} V_G:
    // on a tile whose mesh moves they are interpolated like the others; on a
    // tile where no node moves their departure point is the node itself and
    // they are stored as collided.
    const bool tile_moves = __syncthreads_or(mv) != 0;

    // ---- phase 2: tile+2: D_a = (mu/p) d_{x_a} dQ_a --------------------------
    for (int e = t; e < R2N; e += K1_THREADS) {
        const int u2 = e % R2X, v2 = e / R2X;
        const int ig = i0 - 2 + u2, jg = j0 - 2 + v2;
        if (!node_exists(P, ig, jg, cg)) {
            sm.D[e] = make_float2(0.0f, 0.0f);
            continue;
        }
        const Sten js = jstencil(P, ig, jg, cg), is = istencil(P, ig, cg);
        const int c = (v2 + 1) * R3X + (u2 + 1);    // R3 index
        float J[4];
        metric(sm, c, is, js, false, J);
        const float idet = rcpf(J[0] * J[3] - J[2] * J[1]);
        const float qx_xi = dsten(sm.u.q.Qx, c, 1, is);
        const float qy_xi = dsten(sm.u.q.Qy, c, 1, is);
        const float qx_eta = dsten(sm.u.q.Qx, c, R3X, js);
        const float qy_eta = dsten(sm.u.q.Qy, c, R3X, js);
        const float s = sm.u.q.S[c] * idet;
        sm.D[e] = make_float2(s * (J[3] * qx_xi - J[2] * qx_eta), s * (-J[1] * qy_xi + J[0] * qy_eta));
    }
    __syncthreads();

    // ---- phase 3: tile+1: F_a = d_{x_a} D_a, collide -> LDS ------------------
#pragma unroll
    for (int rd = 0; rd < R1_ROUNDS; ++rd) {
        const int e = rd * K1_THREADS + t;           // R1 index (= phase-1 item)
        if (e >= R1N) break;
        const int u1 = e % R1X, v1 = e / R1X;
        const int ig = i0 - 1 + u1, jg = j0 - 1 + v1;
        if (!node_exists(P, ig, jg, cg)) continue;
        if (cg && jg < 0) {
            // row -1 across the cut: the exported row-1 state of the mirrored
            // column (only cut columns and duplicated wall points are ever
            // interpolated from)
            if constexpr (!EXPORT) {
                const int slot = cut_slot(P, mirror_col(P, P.exits ? ig : wrap(ig, ni)));
                if (slot >= 0) {
#pragma unroll
                    for (int k = 1; k < 9; ++k)
                        sm.u.FG[e][k] = make_float2(P.cutbuf[(k - 1) * P.cut_n + slot],
                                                    P.cutbuf[(7 + k) * P.cut_n + slot]);
                    if (tile_moves)
                        sm.u.FG[e][0] = make_float2(P.cutbuf[NMOV * P.cut_n + slot],
                                                    P.cutbuf[(NMOV + 1) * P.cut_n + slot]);
                }
            }
            continue;
        }
        const Sten js = jstencil(P, ig, jg, cg), is = istencil(P, ig, cg);
        float J[4];
        metric(sm, (v1 + 2) * R3X + (u1 + 2), is, js, false, J);
        const float idet = rcpf(J[0] * J[3] - J[2] * J[1]);
        const int c = (v1 + 1) * R2X + (u1 + 1);     // R2 index
        const float *Dx = &sm.D[0].x;                // interleaved (x, y): stride 2 floats
        const float dx_xi = dsten(Dx, 2 * c, 2, is), dy_xi = dsten(Dx + 1, 2 * c, 2, is);
        const float dx_eta = dsten(Dx, 2 * c, 2 * R2X, js), dy_eta = dsten(Dx + 1, 2 * c, 2 * R2X, js);
        float Fx = idet * (J[3] * dx_xi - J[2] * dx_eta);
        float Fy = idet * (-J[1] * dy_xi + J[0] * dy_eta);
        // duplicated wall points (both copies): no correction, so that the
        // two copies of the one node collide identically
        if (cg && jg == 0 && dup_point(P, P.exits ? ig : wrap(ig, ni))) {
            Fx = 0.0f;
            Fy = 0.0f;
        }
        float f[9], g[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            f[k] = fk[rd][k];
            g[k] = gk[rd][k];
        }
        collide(f, g, Fx, Fy, P, err);
#pragma unroll
        for (int k = 1; k < 9; ++k) sm.u.FG[e][k] = make_float2(f[k], g[k]);
        if (tile_moves) sm.u.FG[e][0] = make_float2(f[0], g[0]);
        const bool own = u1 >= 1 && u1 <= TILE_X && v1 >= 1 && v1 <= TILE_Y &&
                         i0 + u1 - 1 < ni && j0 + v1 - 1 < nj;
        if constexpr (EXPORT) {
            // row-1 state of the cut columns for the tiles across the cut
            const int slot = cut_slot(P, P.exits ? ig : wrap(ig, ni));
            if (own && jg == 1 && slot >= 0) {
#pragma unroll
                for (int k = 1; k < 9; ++k) {
                    P.cutbuf[(k - 1) * P.cut_n + slot] = f[k];
                    P.cutbuf[(7 + k) * P.cut_n + slot] = g[k];
                }
                P.cutbuf[NMOV * P.cut_n + slot] = f[0];
                P.cutbuf[(NMOV + 1) * P.cut_n + slot] = g[0];
            }
        } else if (own && !tile_moves) {
            // no node of the tile moves: the rest populations stay at their
            // node (a node of the tile itself: 0 <= ig < ni)
            const int off = pop_off<STORE>(jg * ni + ig);
            pop_st<STORE, NT>(P, dst, 0, off, f[0]);
            pop_st<STORE, NT>(P, dst, Q, off, g[0]);
        }
    }
    if constexpr (EXPORT) {
        if (err) atomicOr(P.err, err);
        return;
    }
    __syncthreads();

    // ---- phase 4: tile: departure points + interpolation ---------------------
    const float dtf = P.dt;
    const float inv_dt = rcpf(dtf);
    for (int e = t; e < TILE_X * TILE_Y; e += K1_THREADS) {
        const int ut = e % TILE_X, vt = e / TILE_X;
        const int ig = i0 + ut, jg = j0 + vt;
        if (ig >= ni || jg >= nj) continue;
        // far-field row and C-grid exit columns: boundary kernel
        if (!P.periodic_j && jg == nj - 1) continue;
        if (cg && P.exits && (ig == 0 || ig == ni - 1)) continue;
        const int c3 = (vt + 3) * R3X + (ut + 3);
        const bool wall = !P.periodic_j && jg == 0 && wall_col(P, ig, cg);
        const Sten js = jstencil(P, ig, jg, cg);
        NodeGeo ng;
        // metric of the mesh at t^{n+1}
        metric(sm, c3, centred_sten(), js, true, ng.J);
        // undeformed neighbourhood relative to the node: the four edges out of
        // it (+i, -i, +j, -j) and the far corners of its four cells
        const float2 Xc = sm.Xu[c3];
        ng.Epi = rel_pos(sm, c3 + 1, Xc);
        ng.Emi = rel_pos(sm, c3 - 1, Xc);
        ng.Epj = rel_pos(sm, c3 + R3X, Xc);
        ng.Emj = rel_pos(sm, c3 - R3X, Xc);
        ng.Kpp = rel_pos(sm, c3 + R3X + 1, Xc);
        ng.Kmp = rel_pos(sm, c3 + R3X - 1, Xc);
        ng.Kmm = rel_pos(sm, c3 - R3X - 1, Xc);
        ng.Kpm = rel_pos(sm, c3 - R3X + 1, Xc);
        ng.E2 = wall ? rel_pos(sm, c3 + 2 * R3X, Xc) : make_float2(0.0f, 0.0f);
        // mesh velocity V_G = (x^{n+1} - x^n)/dt
        ng.VGx = sm.dd[c3].x * inv_dt;
        ng.VGy = sm.dd[c3].y * inv_dt;
        uint16_t miss = 0, amb = 0;
        node_stream<STORE, R1X, false, NT>(P, dst, pop_off<STORE>(jg * ni + ig), ng, wall, tile_moves,
                                sm.u.FG, (vt + 1) * R1X + (ut + 1), dtf, miss, amb, err);
        if (wall) {
            P.wall_mask[ig] = miss;
            P.wall_amb[ig] = amb & (uint16_t)~miss;
        }
    }
    if (err) atomicOr(P.err, err);
}

template <int STORE, bool CG, int TX, int TY, bool NT = false>
__global__ void __launch_bounds__(TX * TY, kWavesPerSimd)
k_collide_stream(const Inst *__restrict__ insts, const int2 *__restrict__ work, int n_work) {
    __shared__ K1Smem<Geo<TX, TY>> sm;
    // Work distribution: consecutive dispatch slots go round-robin over the 8
    // XCDs, so each XCD owns a contiguous run of work items (neighbouring tiles
    // share halos in that XCD's L2).  A grid smaller than the item count makes
    // the kernel persistent: each workgroup strides over its XCD's run.
    const int per_xcd = (n_work + 7) / 8;
    const int xcd = blockIdx.x % 8, nloc = gridDim.x / 8;
    for (int li = blockIdx.x / 8; li < per_xcd; li += nloc) {
        const int wk = xcd * per_xcd + li;
        if (wk >= n_work) break;
        const int2 w = work[wk];
        collide_stream_tile<STORE, false, CG, TX, TY, NT>(sm, insts, make_int2(uniform(w.x), uniform(w.y)));
        __syncthreads();                      // LDS is reused by the next item
    }
}

// C-grid pre-pass: one workgroup per tile of row block 0 that holds cut columns
template <int STORE>
__global__ void __launch_bounds__(TILE_X * TILE_Y, kWavesPerSimd)
k_cut_export(const Inst *__restrict__ insts, const int2 *__restrict__ work, int n_work) {
    __shared__ K1Smem<Geo<TILE_X, TILE_Y>> sm;
    if ((int)blockIdx.x >= n_work) return;
    const int2 w = work[blockIdx.x];
    collide_stream_tile<STORE, true, true, TILE_X, TILE_Y>(sm, insts, make_int2(uniform(w.x), uniform(w.y)));
}

// ---------------------------------------------------------------------------
// Boundary kernels (O-grid).  Work items (instance, block): 64 wall or
// far-field nodes per block.
// ---------------------------------------------------------------------------
constexpr int BND = 64;

// quadratic Lagrange basis on the nodes {-1, 0, +1}
template <typename R>
__device__ __forceinline__ R lag(int p, R a) {
    return p < 0 ? R(0.5) * a * (a - R(1)) : (p == 0 ? R(1) - a * a : R(0.5) * a * (a + R(1)));
}

template <int STORE>
__device__ __forceinline__ void load_node(const Inst &P, const void *base, long long idx, float f[9],
                                          float g[9]) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        f[k] = pop_load<STORE>(P, base, k, idx);
        g[k] = pop_load<STORE>(P, base, Q + k, idx);
    }
}

// physical position of node idx at the level whose body states are s[] (FP64):
// every body moves the nodes of its own region of influence
__device__ __forceinline__ void node_pos(const Inst &P, long long idx, const BodySlot *s, double &x,
                                         double &y) {
    const double2 X = P.X[idx];
    x = X.x;
    y = X.y;
    for (int k = 0; k < P.nbody; ++k) {
        const double r = blend_factor(P, k, idx, X.x, X.y);
        if (r < 1.0) {
            double dx, dy;
            rigid_disp(P.body[k], s[k], X.x, X.y, dx, dy);
            x += (1.0 - r) * dx;
            y += (1.0 - r) * dy;
        }
    }
}

// wall block blk (BND columns of one wall segment): its segment and first
// column; false past the last block
__device__ __forceinline__ bool wall_block(const Inst &P, int blk, int &seg, int &c0) {
    for (int k = 0; k < P.n_seg; ++k) {
        const int nb = (P.seg_n[k] + BND - 1) / BND;
        if (blk < nb) {
            seg = k;
            c0 = P.seg_i0[k] + blk * BND;
            return true;
        }
        blk -= nb;
    }
    return false;
}

// FP64 geometry of wall node ig for the departure points of its populations
// at level n: the metric of x^{n+1} (centred along the wall, one-sided into
// the fluid) and of X, the mesh velocity, and the edges and twist of the two
// first-row cells (toward i - 1 and toward i + 1), in absolute FP64
// coordinates.  The same steps as the collision-streaming kernel's FP32
// evaluation; formed once per node for all its populations.
struct WallDepGeo {
    double idet, j11, j21, j12, j22, b11, b21, b12, b22, vgx, vgy;
    double ejx, ejy, eix[2], eiy[2], twx[2], twy[2];
};

__device__ WallDepGeo wall_departure_geo(const Inst &P, int ig, long long n) {
    const int ni = P.ni;
    const int im = P.exits ? ig - 1 : wrap(ig - 1, ni), ip = P.exits ? ig + 1 : wrap(ig + 1, ni);
    const BodySlot *s0 = P.slots + (n % 3) * MAX_BODIES, *s1 = P.slots + ((n + 1) % 3) * MAX_BODIES;
    const long long i1 = (long long)ni + ig, i2 = 2LL * ni + ig;
    double xm, ym, xp, yp, x0, y0, x1, y1, x2, y2, x0n, y0n;
    node_pos(P, im, s1, xm, ym);
    node_pos(P, ip, s1, xp, yp);
    node_pos(P, ig, s1, x0, y0);
    node_pos(P, i1, s1, x1, y1);
    node_pos(P, i2, s1, x2, y2);
    node_pos(P, ig, s0, x0n, y0n);
    const double2 X0 = P.X[ig], Xm = P.X[im], Xp = P.X[ip], X1 = P.X[i1], X2 = P.X[i2];
    const double2 Xm1 = P.X[(long long)ni + im], Xp1 = P.X[(long long)ni + ip];
    WallDepGeo w;
    w.j11 = 0.5 * (xp - xm);
    w.j21 = 0.5 * (yp - ym);
    w.j12 = 2.0 * (x1 - x0) - 0.5 * (x2 - x0);
    w.j22 = 2.0 * (y1 - y0) - 0.5 * (y2 - y0);
    w.b11 = 0.5 * (Xp.x - Xm.x);
    w.b21 = 0.5 * (Xp.y - Xm.y);
    w.b12 = 2.0 * (X1.x - X0.x) - 0.5 * (X2.x - X0.x);
    w.b22 = 2.0 * (X1.y - X0.y) - 0.5 * (X2.y - X0.y);
    w.vgx = (x0 - x0n) / P.dt_d;
    w.vgy = (y0 - y0n) / P.dt_d;
    w.idet = 1.0 / (w.j11 * w.j22 - w.j12 * w.j21);
    w.ejx = X1.x - X0.x;
    w.ejy = X1.y - X0.y;
    for (int side = 0; side < 2; ++side) {
        const double2 Xs = side ? Xp : Xm, Xs1 = side ? Xp1 : Xm1;
        w.eix[side] = Xs.x - X0.x;
        w.eiy[side] = Xs.y - X0.y;
        w.twx[side] = (Xs1.x - X0.x) - w.eix[side] - w.ejx;
        w.twy[side] = (Xs1.y - X0.y) - w.eiy[side] - w.ejy;
    }
    return w;
}

// FP64 bilinear coordinate v (in units of the first cell row, 0 on the wall
// line) of the departure point of population k at the wall node of `w`: the
// linear departure offset mapped to the undeformed frame, then the bilinear
// inverse of the first-row cell whose i-range holds the point.  Used for the
// populations whose FP32 v lies within reach of the line at which a population
// counts as missing.
__device__ double wall_departure_v(const Inst &P, const WallDepGeo &w, int k) {
    const double wx = (double)CXK(k) - w.vgx, wy = (double)CYK(k) - w.vgy;
    const double ax = -P.dt_d * w.idet * (w.j22 * wx - w.j12 * wy);
    const double ay = -P.dt_d * w.idet * (-w.j21 * wx + w.j11 * wy);
    const double px = w.b11 * ax + w.b12 * ay, py = w.b21 * ax + w.b22 * ay;
    double v_best = 0.0, u_err = 1e300;
    for (int side = 0; side < 2; ++side) {
        const double eix = w.eix[side], eiy = w.eiy[side], ejx = w.ejx, ejy = w.ejy;
        const double twx = w.twx[side], twy = w.twy[side];
        double u = 0.0, v = 0.0;
        for (int it = 0; it < 30; ++it) {   // Newton on u e_i + v e_j + u v tw = p
            const double rx = u * eix + v * ejx + u * v * twx - px;
            const double ry = u * eiy + v * ejy + u * v * twy - py;
            const double jux = eix + v * twx, juy = eiy + v * twy;
            const double jvx = ejx + u * twx, jvy = ejy + u * twy;
            const double d = jux * jvy - juy * jvx;
            const double du = (jvy * rx - jvx * ry) / d, dv = (-juy * rx + jux * ry) / d;
            u -= du;
            v -= dv;
            if (fabs(du) + fabs(dv) < 1e-15) break;
        }
        const double e = u < 0.0 ? -u : (u > 1.0 ? u - 1.0 : 0.0);   // distance outside [0, 1]
        if (e < u_err) {
            u_err = e;
            v_best = v;
        }
    }
    return v_best;
}

// Wall targets (Grad BC, Sec. III.A.1) for item.y even, far-field
// equilibria (Sec. III.A.2) for item.y odd; item.y >> 1 is the block of 64
// wall nodes (of one wall segment) or of 64 far-field list entries.
//   rho_t, T_t : values at B (distance dt along the wall normal), 9-node
//                Lagrange element centred on row 1; the wall row of the
//                element holds the previous step's values
//   u_t        : mesh velocity of the wall node (no slip on a moving wall)
template <int STORE>
__global__ void __launch_bounds__(BND) k_wall_targets(const Inst *__restrict__ insts,
                                                      const int2 *__restrict__ work, int n_work) {
    __shared__ float s_rho[3][BND + 2], s_T[3][BND + 2];
    if ((int)blockIdx.x >= n_work) return;
    const int2 item = work[blockIdx.x];
    const Inst &P = insts[item.x];
    const int kind = item.y & 1, blk = item.y >> 1;
    const long long n = *P.step;
    const void *src = P.pop[n & 1];
    void *dst = P.pop[(n + 1) & 1];
    const int ni = P.ni, t = threadIdx.x;
    if (kind == 0) {
        int seg, i0;
        if (!wall_block(P, blk, seg, i0)) return;
        const int iend = P.seg_i0[seg] + P.seg_n[seg];
        const int ig = i0 + t, igc = min(ig, iend - 1);
        // this node's inputs, requested with the element's populations: the
        // rows 0 (previous level), 1 and 2 of columns i0 - 1 .. i0 + BND, every
        // load of this thread's items in flight together (the lanes past the
        // end repeat the last item)
        const uint16_t amb = P.wall_amb[igc];
        const float2 B = P.wall_B[igc];
        const double2 X = P.X[igc];
        constexpr int NS = 3 * (BND + 2), NE = (NS + BND - 1) / BND;
        float fe[NE][9], ge[NE][9];
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int e = min(t + q * BND, NS - 1);
            const int r = e / (BND + 2), c = e % (BND + 2);
            load_node<STORE>(P, r == 0 ? src : dst, (long long)r * ni + wrap(i0 - 1 + c, ni), fe[q], ge[q]);
        }
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int e = t + q * BND;
            if (e < NS) {
                const Moments m = moments(fe[q], ge[q], P.Cv);
                s_rho[e / (BND + 2)][e % (BND + 2)] = m.rho;
                s_T[e / (BND + 2)][e % (BND + 2)] = m.T;
            }
        }
        __syncthreads();
        if (ig >= iend) return;
        // missing or not, decided in FP64 where the FP32 evaluation was too close to call
        if (amb) {
            uint16_t miss = P.wall_mask[ig];
            const WallDepGeo wd = wall_departure_geo(P, ig, n);
            for (int k = 0; k < 9; ++k)
                if ((amb & (1u << k)) && wall_departure_v(P, wd, k) < -1e-4) miss |= (uint16_t)(1u << k);
            P.wall_mask[ig] = miss;
        }
        const float a = B.x, b = B.y - 1.0f;   // offsets from the element centre (i, 1)
        float rho_t = 0.0f, T_t = 0.0f;
#pragma unroll
        for (int q = -1; q <= 1; ++q)
#pragma unroll
            for (int p = -1; p <= 1; ++p) {
                const float w = lag(p, a) * lag(q, b);
                rho_t += w * s_rho[q + 1][t + 1 + p];
                T_t += w * s_T[q + 1][t + 1 + p];
            }
        double vx = 0.0, vy = 0.0;
        const BodySlot *s1 = P.slots + ((n + 1) % 3) * MAX_BODIES, *s0 = P.slots + (n % 3) * MAX_BODIES;
        for (int k = 0; k < P.nbody; ++k) {
            const double r = blend_factor(P, k, ig, X.x, X.y);
            if (r < 1.0) {
                double d1x, d1y, d0x, d0y;
                rigid_disp(P.body[k], s1[k], X.x, X.y, d1x, d1y);
                rigid_disp(P.body[k], s0[k], X.x, X.y, d0x, d0y);
                vx += (1.0 - r) * (d1x - d0x) / P.dt_d;
                vy += (1.0 - r) * (d1y - d0y) / P.dt_d;
            }
        }
        P.wall_tgt[ig] = make_float4(rho_t, (float)vx, (float)vy, T_t);
    } else {
        const int k = blk * BND + t;
        if (k >= P.n_ff) return;
        const int2 node = P.ff[k];             // (far-field node, interior node)
        float rho, ux, uy, T;
        if (P.inflow[k]) {
            rho = P.rho_inf; ux = P.ux_inf; uy = P.uy_inf; T = P.T_inf;
        } else {  // outlet: zero gradient, copy the adjacent interior node
            float f[9], g[9];
            load_node<STORE>(P, dst, node.y, f, g);
            const Moments m = moments(f, g, P.Cv);
            rho = m.rho; ux = m.ux; uy = m.uy; T = m.T;
        }
        const float E = P.Cv * T + 0.5f * (ux * ux + uy * uy);
        float feq[9], geq[9];
        equilibria<float>(rho, ux, uy, T, E, feq, geq);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            pop_store<STORE>(P, dst, q, node.x, feq[q]);
            pop_store<STORE>(P, dst, Q + q, node.x, geq[q]);
        }
    }
}

// Tangential neighbour values (ux, uy, T) for the wall-gradient stencil: the
// neighbour's target if it is a wall node, else (a C-grid cut node next to the
// trailing edge) its freshly streamed state.
template <int STORE>
__device__ __forceinline__ float4 wall_neighbour(const Inst &P, const void *buf, int i) {
    if (wall_col(P, i)) return P.wall_tgt[i];
    float f[9], g[9];
    load_node<STORE>(P, buf, i, f, g);
    const Moments m = moments(f, g, P.Cv);
    return make_float4(m.rho, m.ux, m.uy, m.T);
}

// Grad populations (Sec. III.A.1) for the missing populations of wall node ig
// of the level in `buf`: f, g enter as loaded and leave with the missing ones
// replaced (unrounded).
template <int STORE>
__device__ void grad_fill(const Inst &P, const void *buf, const BodySlot *sL, int ig, float f[9],
                          float g[9]) {
    const uint16_t miss = P.wall_mask[ig];
    if (!miss) return;
    const int ni = P.ni;
    const int im = P.exits ? ig - 1 : wrap(ig - 1, ni), ip = P.exits ? ig + 1 : wrap(ig + 1, ni);
    double xm, ym, xp, yp, x0, y0;
    node_pos(P, im, sL, xm, ym);
    node_pos(P, ip, sL, xp, yp);
    node_pos(P, ig, sL, x0, y0);
    const float Cv = P.Cv, Cp = P.Cp, dt = P.dt;
    const float4 tm = wall_neighbour<STORE>(P, buf, im), t0 = P.wall_tgt[ig];
    const float4 tp = wall_neighbour<STORE>(P, buf, ip);
    float f1[9], g1[9], f2[9], g2[9];
    load_node<STORE>(P, buf, (long long)ni + ig, f1, g1);
    load_node<STORE>(P, buf, 2LL * ni + ig, f2, g2);
    const Moments m1 = moments(f1, g1, Cv), m2 = moments(f2, g2, Cv);
    // metric of the mesh at t^{n+1} at the wall node: centred along the
    // wall, one-sided into the fluid
    double x1, y1, x2, y2;
    node_pos(P, (long long)ni + ig, sL, x1, y1);
    node_pos(P, 2LL * ni + ig, sL, x2, y2);
    const float x_xi = (float)(0.5 * (xp - xm)), y_xi = (float)(0.5 * (yp - ym));
    const float x_eta = (float)(2.0 * (x1 - x0) - 0.5 * (x2 - x0));
    const float y_eta = (float)(2.0 * (y1 - y0) - 0.5 * (y2 - y0));
    const float idet = 1.0f / (x_xi * y_eta - y_xi * x_eta);
    const float rho_t = t0.x, ux_t = t0.y, uy_t = t0.z, T_t = t0.w;
    const float E_t = Cv * T_t + 0.5f * (ux_t * ux_t + uy_t * uy_t);
    const float Em = Cv * tm.w + 0.5f * (tm.y * tm.y + tm.z * tm.z);
    const float Ep = Cv * tp.w + 0.5f * (tp.y * tp.y + tp.z * tp.z);
    const float E1 = Cv * m1.T + 0.5f * (m1.ux * m1.ux + m1.uy * m1.uy);
    const float E2 = Cv * m2.T + 0.5f * (m2.ux * m2.ux + m2.uy * m2.uy);
    // (C_xi, C_eta) -> (dC/dx, dC/dy)
    auto grad = [&](float cm, float c0, float cp, float c1, float c2, float &gx, float &gy) {
        const float cxi = 0.5f * (cp - cm);
        const float ceta = -1.5f * c0 + 2.0f * c1 - 0.5f * c2;
        gx = idet * (y_eta * cxi - y_xi * ceta);
        gy = idet * (-x_eta * cxi + x_xi * ceta);
    };
    float duxx, duxy, duyx, duyy, dTx, dTy, dEx, dEy;
    grad(tm.y, ux_t, tp.y, m1.ux, m2.ux, duxx, duxy);
    grad(tm.z, uy_t, tp.z, m1.uy, m2.uy, duyx, duyy);
    grad(tm.w, T_t, tp.w, m1.T, m2.T, dTx, dTy);
    grad(Em, E_t, Ep, E1, E2, dEx, dEy);
    grad_populations(P, miss, rho_t, ux_t, uy_t, T_t, E_t, duxx, duxy, duyx, duyy, dTx, dTy, dEx, dEy,
                     f, g);
}

// Grad populations for the missing wall populations (phase 1 only) and the
// traction F_k = sigma . (n ds)_k of every node of each body's wall polygon at
// the current level (Sec. III: sigma = -p I - (1 - omega/2) P^(1),
// P^(1) = sum (f - f^eq) c c; (n ds)_k = 1/2 rot_{+90}(x_{k+1} - x_{k-1}) with
// k +- 1 the polygon neighbours).  A wall segment that ends on a second copy
// of its first point (a C-grid's trailing edge, a twin O-grid's junctions):
// both copies are filled, and the thread of the first copy stores one merged
// state in both: population by population the streamed value of the copy that
// found its departure point, else the mean of the two copies.  Blocks of two
// waves: the first takes BND wall nodes; the second, in the block that holds
// the first copy of a duplicated point, fills the second copy meanwhile.
template <int STORE>
__global__ void __launch_bounds__(2 * BND) k_wall_grad_force(const Inst *__restrict__ insts,
                                                             const int2 *__restrict__ work, int n_work,
                                                             int phase) {
    __shared__ float s_fu[9], s_gu[9];        // second copy, Grad-filled
    if ((int)blockIdx.x >= n_work) return;
    const int2 item = work[blockIdx.x];
    const Inst &P = insts[item.x];
    int seg, c0;
    if (!wall_block(P, item.y, seg, c0)) return;
    const int w0 = P.seg_i0[seg], dup = P.seg_dup[seg];
    const int te_up = w0 + P.seg_n[seg] - 1;
    const bool pair = phase && dup && c0 == w0;   // the same for the whole block
    const long long n = *P.step;
    const long long L = phase ? n + 1 : n;
    void *buf = P.pop[L & 1];
    const BodySlot *sL = P.slots + (L % 3) * MAX_BODIES;
    if (threadIdx.x >= BND) {
        if (pair) {
            if (threadIdx.x == BND) {
                float fu[9], gu[9];
                load_node<STORE>(P, buf, te_up, fu, gu);
                grad_fill<STORE>(P, buf, sL, te_up, fu, gu);
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    s_fu[k] = fu[k];
                    s_gu[k] = gu[k];
                }
            }
            __syncthreads();
        }
        return;
    }
    const int ig = c0 + threadIdx.x;
    // a node of this block (the second copy goes with the first)
    const bool live = ig < w0 + P.seg_n[seg] && !(dup && ig == te_up);
    if (!live && !pair) return;
    // positions for the traction's normal (polygon neighbours), formed while
    // the populations load
    const int fn = P.seg_n[seg] - dup;       // distinct nodes of the polygon
    const int fm = ig == w0 ? w0 + fn - 1 : ig - 1;
    const int fp = ig == w0 + fn - 1 ? w0 : ig + 1;
    double xm = 0.0, ym = 0.0, xp = 0.0, yp = 0.0, x0 = 0.0, y0 = 0.0;
    float f[9], g[9];
    if (live) {
        node_pos(P, fm, sL, xm, ym);
        node_pos(P, fp, sL, xp, yp);
        node_pos(P, ig, sL, x0, y0);
        load_node<STORE>(P, buf, ig, f, g);
        if (phase) grad_fill<STORE>(P, buf, sL, ig, f, g);
    }
    if (pair) __syncthreads();
    if (!live) return;
    if (phase) {
        if (pair && ig == w0) {
            const unsigned ml = P.wall_mask[ig], mu = P.wall_mask[te_up];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const float fu = s_fu[k], gu = s_gu[k];
                const bool lo_miss = ml & (1u << k), up_miss = mu & (1u << k);
                f[k] = (lo_miss && !up_miss) ? fu : ((up_miss && !lo_miss) ? f[k] : 0.5f * (f[k] + fu));
                g[k] = (lo_miss && !up_miss) ? gu : ((up_miss && !lo_miss) ? g[k] : 0.5f * (g[k] + gu));
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                pop_store<STORE>(P, buf, k, ig, f[k]);
                pop_store<STORE>(P, buf, Q + k, ig, g[k]);
                pop_store<STORE>(P, buf, k, te_up, f[k]);
                pop_store<STORE>(P, buf, Q + k, te_up, g[k]);
                f[k] = pop_round<STORE>(P, k, f[k]);
                g[k] = pop_round<STORE>(P, Q + k, g[k]);
            }
        } else if (P.wall_mask[ig]) {
            const unsigned miss = P.wall_mask[ig];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                if (!(miss & (1u << k))) continue;
                pop_store<STORE>(P, buf, k, ig, f[k]);
                pop_store<STORE>(P, buf, Q + k, ig, g[k]);
                // the traction below sees the populations as stored
                f[k] = pop_round<STORE>(P, k, f[k]);
                g[k] = pop_round<STORE>(P, Q + k, g[k]);
            }
        }
    }
    // traction of the complete wall node, with the moments formed in FP64
    // from the stored populations; normals from the polygon neighbours
    double sxx, sxy, syy;
    const bool ok = wall_stress(P, f, g, sxx, sxy, syy);
    const double nx = -0.5 * (yp - ym), ny = 0.5 * (xp - xm);
    const double Fx = sxx * nx + sxy * ny;
    const double Fy = sxy * nx + syy * ny;
    const double rx = x0 - P.body[seg].ex, ry = y0 - (P.body[seg].ey + sL[seg].h);
    P.wall_force[ig] = make_double4(Fx, Fy, rx * Fy - ry * Fx, 0.0);
    if (!ok) atomicOr(P.err, ERR_STATE);
}

// ---------------------------------------------------------------------------
// Rigid body (Sec. IV): fixed-order FP64 traction sum, RK4 with the load
// frozen over the step, or the prescribed motion.  One block per instance.
// ---------------------------------------------------------------------------
__device__ void body_accel(const Body &b, double h, double a, double Fy, double M, double &hdd,
                           double &add) {
    if (b.dof == DOF_HEAVE) {
        hdd = (Fy - b.k_h * h) / b.m;
        add = 0.0;
    } else {  // pitch-plunge: [m S; S I] [h''; a''] = [Fy - k_h h; M - k_a a]
        const double r1 = Fy - b.k_h * h, r2 = M - b.k_a * a;
        const double det = b.m * b.I_a - b.S_a * b.S_a;
        hdd = (b.I_a * r1 - b.S_a * r2) / det;
        add = (-b.S_a * r1 + b.m * r2) / det;
    }
}

// state at t^{n+1} from s at t^n: the prescribed motion, or RK4 of the body
// equation with the load varying linearly from (Fy, M) at t^n to (Fy1, M1) at
// t^{n+1} (equal for the staggered step, whose load is frozen)
__device__ BodySlot body_advance(const Body &b, const BodySlot &s, double Fy, double M, double Fy1,
                                 double M1, double t_next, double dt) {
    BodySlot o = s;
    const bool forced = (b.dof == DOF_HEAVE || b.dof == DOF_PITCH_PLUNGE) && b.release_time > 0.0 &&
                        t_next <= b.release_time;
    if (b.present && (b.dof == DOF_PRESCRIBED || forced)) {
        o.h = b.heave_amp * sin(b.heave_omega * t_next);
        o.hd = b.heave_amp * b.heave_omega * cos(b.heave_omega * t_next);
        o.a = b.pitch_amp * sin(b.pitch_omega * t_next);
        o.ad = b.pitch_amp * b.pitch_omega * cos(b.pitch_omega * t_next);
    } else if (b.present && (b.dof == DOF_HEAVE || b.dof == DOF_PITCH_PLUNGE)) {
        double y[4] = {s.h, s.a, s.hd, s.ad}, k[4][4];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const double c = st == 0 ? 0.0 : (st == 3 ? dt : 0.5 * dt);
            double z[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) z[q] = st == 0 ? y[q] : y[q] + c * k[st - 1][q];
            double hdd, add;
            body_accel(b, z[0], z[1], Fy + c / dt * (Fy1 - Fy), M + c / dt * (M1 - M), hdd, add);
            k[st][0] = z[2];
            k[st][1] = z[3];
            k[st][2] = hdd;
            k[st][3] = add;
        }
        o.h = y[0] + dt / 6.0 * (k[0][0] + 2.0 * k[1][0] + 2.0 * k[2][0] + k[3][0]);
        o.a = y[1] + dt / 6.0 * (k[0][1] + 2.0 * k[1][1] + 2.0 * k[2][1] + k[3][1]);
        o.hd = y[2] + dt / 6.0 * (k[0][2] + 2.0 * k[1][2] + 2.0 * k[2][2] + k[3][2]);
        o.ad = y[3] + dt / 6.0 * (k[0][3] + 2.0 * k[1][3] + 2.0 * k[2][3] + k[3][3]);
    }
    const double sh = sin(0.5 * o.a);
    o.cm1 = -2.0 * sh * sh;
    o.sa = sin(o.a);
    return o;
}

constexpr int BODY_THREADS = 1024;

// Row 0 of the cut: the mirror copy of each primary cut node (columns
// cut_a < c < cut_b) takes its populations (stored words copied as they are),
// on the body kernel's threads t >= 0 of MIRROR_THREADS.  The primary and
// mirror columns are distinct, so every thread issues the loads of eight
// items before any of their stores.
constexpr int MIRROR_THREADS = BODY_THREADS - 64 * MAX_BODIES;

template <typename W>
__device__ void mirror_cut_row(const Inst &P, W *buf, int t) {
    constexpr int U = 8;
    const int np = P.cut_b - P.cut_a - 1, total = NPOP * np;
    for (int e0 = t; e0 < total; e0 += U * MIRROR_THREADS) {
        W v[U];
        long long to[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = min(e0 + u * MIRROR_THREADS, total - 1);
            const int q = e / np, c = P.cut_a + 1 + e % np;
            const int m = P.exits ? P.mirror - c : wrap(P.mirror - c, P.ni);
            v[u] = buf[(long long)q * P.n_nodes + c];
            to[u] = (long long)q * P.n_nodes + m;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e0 + u * MIRROR_THREADS < total) buf[to[u]] = v[u];
    }
}

__global__ void __launch_bounds__(BODY_THREADS) k_body(const Inst *__restrict__ insts, int phase) {
    constexpr int NW = BODY_THREADS / 64;
    __shared__ double sx[MAX_BODIES][NW], sy[MAX_BODIES][NW], sz[MAX_BODIES][NW];
    const Inst &P = insts[blockIdx.x];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const long long n = *P.step;
    const long long L = phase ? n + 1 : n;
    // the load of every body: the traction sum over its wall polygon, in a
    // fixed order (per thread a stride of the polygon, loads issued four at a
    // time for every polygon together; then the lanes of each wave pairwise;
    // then the waves in order)
    const int nseg = min(P.n_seg, MAX_BODIES);
    int fn[MAX_BODIES], fn_max = 0;
    const double4 *wf[MAX_BODIES];
#pragma unroll
    for (int k = 0; k < MAX_BODIES; ++k) {
        fn[k] = k < nseg ? P.seg_n[k] - P.seg_dup[k] : 0;
        wf[k] = P.wall_force + (k < nseg ? P.seg_i0[k] : 0);
        fn_max = max(fn_max, fn[k]);
    }
    double fx[MAX_BODIES] = {}, fy[MAX_BODIES] = {}, mz[MAX_BODIES] = {};
    for (int i0 = t; i0 < fn_max; i0 += 4 * BODY_THREADS) {
        double4 v[MAX_BODIES][4];
#pragma unroll
        for (int k = 0; k < MAX_BODIES; ++k)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u * BODY_THREADS;
                v[k][u] = i < fn[k] ? wf[k][i] : make_double4(0.0, 0.0, 0.0, 0.0);
            }
#pragma unroll
        for (int k = 0; k < MAX_BODIES; ++k)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                fx[k] += v[k][u].x;
                fy[k] += v[k][u].y;
                mz[k] += v[k][u].z;
            }
    }
#pragma unroll
    for (int k = 0; k < MAX_BODIES; ++k) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            fx[k] += __shfl_down(fx[k], o, 64);
            fy[k] += __shfl_down(fy[k], o, 64);
            mz[k] += __shfl_down(mz[k], o, 64);
        }
        if (lane == 0) {
            sx[k][wv] = fx[k];
            sy[k][wv] = fy[k];
            sz[k][wv] = mz[k];
        }
    }
    __syncthreads();
    double F[MAX_BODIES][3] = {};
#pragma unroll
    for (int k = 0; k < MAX_BODIES; ++k) {
        if (k >= nseg) break;
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int w = 0; w < NW; ++w) {
            ax += sx[k][w];
            ay += sy[k][w];
            az += sz[k][w];
        }
        F[k][0] = ax;
        F[k][1] = ay;
        F[k][2] = az;
    }
    if (wv >= MAX_BODIES) {
        if (phase == 1 && P.cut) {
            // one state per cut point: the mirror copy of each primary cut
            // node takes its populations (duplicated wall points are merged at
            // the wall); the waves that do not advance a body
            void *buf = P.pop[(n + 1) & 1];
            if (P.storage)
                mirror_cut_row<uint16_t>(P, static_cast<uint16_t *>(buf), t - 64 * MAX_BODIES);
            else
                mirror_cut_row<uint32_t>(P, static_cast<uint32_t *>(buf), t - 64 * MAX_BODIES);
        }
        return;
    }
    const int nrec = P.nbody > 0 ? P.nbody : 1;
    if (phase == 2 || (phase == 1 && P.n_sub > 1)) {
        // strong coupling (thread 0): the structure re-solved over step
        // n -> n+1 with the load varying linearly from F^n (the record of
        // level n) to the load of the new populations; a sub-iteration relaxes
        // the estimate of level n+1 towards it, the last one only measures the
        // remaining change
        if (t == 0) {
            const BodySlot *sn = P.slots + (n % 3) * MAX_BODIES;
            BodySlot *s1 = P.slots + ((n + 1) % 3) * MAX_BODIES;
            BodySlot target[MAX_BODIES];
#pragma unroll
            for (int m = 0; m < MAX_BODIES; ++m) {
                if (m >= nrec) break;
                if (P.body[m].master != m) continue;
                double fy0 = 0.0, mz0 = 0.0, fy1 = 0.0, mz1 = 0.0;
#pragma unroll
                for (int k = 0; k < MAX_BODIES; ++k) {
                    if (k >= nrec) break;
                    if (P.body[k].master != m) continue;
                    const double *rec = P.history + ((size_t)k * HIST_CAP + (size_t)(n % HIST_CAP)) * 6;
                    fy0 += rec[2];
                    mz0 += rec[3];
                    fy1 += F[k][1];
                    mz1 += F[k][2];
                }
                target[m] = body_advance(P.body[m], sn[m], fy0, mz0, fy1, mz1, (double)(n + 1) * P.dt_d,
                                         P.dt_d);
            }
#pragma unroll
            for (int k = 0; k < MAX_BODIES; ++k) {
                if (k >= nrec) break;
                BodySlot tg = target[0];          // target of its master (a register select)
#pragma unroll
                for (int q = 1; q < MAX_BODIES; ++q)
                    if (P.body[k].master == q) tg = target[q];
                const BodySlot &cur = s1[k];
                P.resid[k] = fmax(fmax(fabs(tg.h - cur.h), fabs(tg.a - cur.a)),
                                  fmax(fabs(tg.hd - cur.hd), fabs(tg.ad - cur.ad)));
            }
            if (phase == 2) {
#pragma unroll
                for (int m = 0; m < MAX_BODIES; ++m) {
                    if (m >= nrec) break;
                    if (P.body[m].master != m) continue;
                    BodySlot o = s1[m];
                    const BodySlot &tg = target[m];
                    const double w = P.relax;
                    o.h += w * (tg.h - o.h);
                    o.a += w * (tg.a - o.a);
                    o.hd += w * (tg.hd - o.hd);
                    o.ad += w * (tg.ad - o.ad);
                    const double sh = sin(0.5 * o.a);
                    o.cm1 = -2.0 * sh * sh;
                    o.sa = sin(o.a);
                    s1[m] = o;
                }
                for (int k = 0; k < nrec; ++k)
                    if (P.body[k].master != k) s1[k] = s1[P.body[k].master];
            }
        }
        if (phase == 2) return;
    }
    // record k on the first lane of wave k: its history entry, and its state
    // at the next level, that of its master body, which takes its own load
    // plus those of the bodies linked to it (frozen over the next step: the
    // staggered scheme, and the predictor of strong coupling); a linked body
    // forms its master's state itself, from the same inputs
    if (lane != 0 || wv >= nrec) return;
    const int k = wv;
    const BodySlot *cur = P.slots + (L % 3) * MAX_BODIES;
    BodySlot *nxt = P.slots + ((L + 1) % 3) * MAX_BODIES;
    double Fk[3] = {F[0][0], F[0][1], F[0][2]};
#pragma unroll
    for (int q = 1; q < MAX_BODIES; ++q)
        if (k == q) {
            Fk[0] = F[q][0];
            Fk[1] = F[q][1];
            Fk[2] = F[q][2];
        }
    double *rec = P.history + ((size_t)k * HIST_CAP + (size_t)(L % HIST_CAP)) * 6;
    rec[0] = (double)L; rec[1] = Fk[0]; rec[2] = Fk[1]; rec[3] = Fk[2];
    rec[4] = cur[k].h; rec[5] = cur[k].a;
    const int m = P.body[k].master;
    double fys = 0.0, mzs = 0.0;
#pragma unroll
    for (int j = 0; j < MAX_BODIES; ++j) {
        if (j >= nrec) break;
        if (P.body[j].master != m) continue;
        fys += F[j][1];
        mzs += F[j][2];
    }
    nxt[k] = body_advance(P.body[m], cur[m], fys, mzs, fys, mzs, (double)(L + 1) * P.dt_d, P.dt_d);
    if (phase && k == 0) *P.step = n + 1;
}

// ---------------------------------------------------------------------------
// initial equilibria, macroscopic dump, storage codec
// ---------------------------------------------------------------------------
template <int STORE>
__global__ void k_init_equilibrium(const Inst *__restrict__ pinst, const double *__restrict__ macro) {
    const Inst &P = *pinst;
    const long long N = P.n_nodes;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < N;
         idx += (long long)gridDim.x * blockDim.x) {
        const double rho = macro[idx], ux = macro[N + idx], uy = macro[2 * N + idx], T = macro[3 * N + idx];
        const double Cv = 1.0 / P.gm1_d;
        const double E = Cv * T + 0.5 * (ux * ux + uy * uy);
        double feq[9], geq[9];
        equilibria<double>(rho, ux, uy, T, E, feq, geq);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            pop_store<STORE>(P, P.pop[0], k, idx, (float)feq[k]);
            pop_store<STORE>(P, P.pop[0], Q + k, idx, (float)geq[k]);
        }
    }
}

template <int STORE>
__global__ void k_dump_macro(const Inst *__restrict__ pinst, int side, double *__restrict__ out) {
    const Inst &P = *pinst;
    const long long N = P.n_nodes;
    const void *src = P.pop[side];
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < N;
         idx += (long long)gridDim.x * blockDim.x) {
        double rho = 0, jx = 0, jy = 0, G = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double fk = pop_load<STORE>(P, src, k, idx);
            rho += fk;
            jx += CXK(k) * fk;
            jy += CYK(k) * fk;
            G += (double)pop_load<STORE>(P, src, Q + k, idx);
        }
        const double ux = jx / rho, uy = jy / rho;
        const double E = 0.5 * G / rho;
        const double T = (E - 0.5 * (ux * ux + uy * uy)) * P.gm1_d;
        out[idx] = rho;
        out[N + idx] = ux;
        out[2 * N + idx] = uy;
        out[3 * N + idx] = T;
    }
}

template <int STORE>
__global__ void k_decode(const Inst *__restrict__ pinst, int side, int q0, float *__restrict__ out) {
    const Inst &P = *pinst;
    const long long N = P.n_nodes;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < 9 * N;
         e += (long long)gridDim.x * blockDim.x) {
        const int q = (int)(e / N);
        out[e] = pop_load<STORE>(P, P.pop[side], q0 + q, e - q * N);
    }
}

template <int STORE>
__global__ void k_encode(const Inst *__restrict__ pinst, int side, int q0, const float *__restrict__ in) {
    const Inst &P = *pinst;
    const long long N = P.n_nodes;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < 9 * N;
         e += (long long)gridDim.x * blockDim.x) {
        const int q = (int)(e / N);
        pop_store<STORE>(P, P.pop[side], q0 + q, e - q * N, in[e]);
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
hipError_t launch_collide_stream(const Inst *insts, const int2 *work, int n_work, int storage,
                                 hipStream_t s, int grid, bool cut, int shape, bool stream_out) {
    // one workgroup per item unless a smaller (persistent) grid is requested;
    // always a multiple of the XCD count
    const int all = ((n_work + 7) / 8) * 8;
    int g = grid > 0 ? ((grid + 7) / 8) * 8 : all;
    if (g > all) g = all;
    if (g < 8) g = 8;
    // the C-grid-capable build (default tile shape only) when some instance of
    // the launch needs it
    if (cut && shape != 0) return hipErrorInvalidValue;
    if (shape < 0 || shape >= N_TILE_SHAPES) return hipErrorInvalidValue;
    const dim3 G(g), B(TILE_SHAPES[shape][0] * TILE_SHAPES[shape][1]);
#define FSI_K1(ST, CGV, TXV, TYV) \
    hipLaunchKernelGGL((k_collide_stream<ST, CGV, TXV, TYV>), G, B, 0, s, insts, work, n_work)
    // non-temporal population stores: built for the wide shape only, the
    // shape of the instances whose step streams more than the cache holds
    static_assert(TILE_SHAPES[WIDE_SHAPE][0] == 64 && TILE_SHAPES[WIDE_SHAPE][1] == 8, "wide shape");
    const bool nt = stream_out && !cut && shape == WIDE_SHAPE;
    if (nt) {
        if (storage == 0)
            hipLaunchKernelGGL((k_collide_stream<0, false, 64, 8, true>), G, B, 0, s, insts, work, n_work);
        else
            hipLaunchKernelGGL((k_collide_stream<1, false, 64, 8, true>), G, B, 0, s, insts, work, n_work);
    } else if (storage == 0) {
        if (cut) FSI_K1(0, true, TILE_X, TILE_Y);
        else if (shape == 1) FSI_K1(0, false, 64, 8);
        else if (shape == 2) FSI_K1(0, false, 16, 32);
        else if (shape == 3) FSI_K1(0, false, 16, 16);
        else FSI_K1(0, false, TILE_X, TILE_Y);
    } else {
        if (cut) FSI_K1(1, true, TILE_X, TILE_Y);
        else if (shape == 1) FSI_K1(1, false, 64, 8);
        else if (shape == 2) FSI_K1(1, false, 16, 32);
        else if (shape == 3) FSI_K1(1, false, 16, 16);
        else FSI_K1(1, false, TILE_X, TILE_Y);
    }
#undef FSI_K1
    return hipGetLastError();
}

hipError_t launch_cut_export(const Inst *insts, const int2 *work, int n_work, int storage,
                             hipStream_t s) {
    FSI_DISPATCH(storage, k_cut_export, dim3(n_work), dim3(TILE_X * TILE_Y), s, insts, work, n_work);
    return hipGetLastError();
}

hipError_t launch_wall_targets(const Inst *insts, const int2 *work, int n_work, int storage,
                               hipStream_t s) {
    FSI_DISPATCH(storage, k_wall_targets, dim3(n_work), dim3(BND), s, insts, work, n_work);
    return hipGetLastError();
}

hipError_t launch_wall_grad_force(const Inst *insts, const int2 *work, int n_work, int storage,
                                  int phase, hipStream_t s) {
    FSI_DISPATCH(storage, k_wall_grad_force, dim3(n_work), dim3(2 * BND), s, insts, work, n_work, phase);
    return hipGetLastError();
}

hipError_t launch_body(const Inst *insts, int n_inst, int phase, hipStream_t s) {
    hipLaunchKernelGGL(k_body, dim3(n_inst), dim3(BODY_THREADS), 0, s, insts, phase);
    return hipGetLastError();
}

static int io_grid(long long n) {
    long long g = (n + 255) / 256;
    return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

hipError_t launch_init_equilibrium(const Inst *inst, const double *macro, long long n_nodes,
                                   int storage, hipStream_t s) {
    FSI_DISPATCH(storage, k_init_equilibrium, dim3(io_grid(n_nodes)), dim3(256), s, inst, macro);
    return hipGetLastError();
}

hipError_t launch_dump_macro(const Inst *inst, int side, double *out, long long n_nodes, int storage,
                             hipStream_t s) {
    FSI_DISPATCH(storage, k_dump_macro, dim3(io_grid(n_nodes)), dim3(256), s, inst, side, out);
    return hipGetLastError();
}

hipError_t launch_decode(const Inst *inst, int side, int q0, float *out, long long n_nodes, int storage,
                         hipStream_t s) {
    FSI_DISPATCH(storage, k_decode, dim3(io_grid(9 * n_nodes)), dim3(256), s, inst, side, q0, out);
    return hipGetLastError();
}

hipError_t launch_encode(const Inst *inst, int side, int q0, const float *in, long long n_nodes,
                         int storage, hipStream_t s) {
    FSI_DISPATCH(storage, k_encode, dim3(io_grid(9 * n_nodes)), dim3(256), s, inst, side, q0, in);
    return hipGetLastError();
}

}  // namespace fsi
