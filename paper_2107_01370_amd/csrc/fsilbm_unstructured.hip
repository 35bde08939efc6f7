// gfx950 kernels of the step on unstructured meshes of 9-node quadrilateral
// elements (Bhadauria, Dorschner & Karlin, arXiv 2107.01370, Sec. II.B on the
// paper's own second-order finite-element meshes).
#include "fsilbm_device.h"
#include "fsilbm_wall.h"

namespace fsi {

// ---------------------------------------------------------------------------
// Unstructured meshes of 9-node quadrilateral elements (Sec. II.B on the
// paper's own finite-element meshes): periodic, or bounded round one body,
// fixed or moving.  Node-wise kernels, data reached through the element
// connectivity:
//   k_u_egrad    element derivatives at the element's nine nodes (of delta Q_a,
//                which the previous step's interpolation formed with mu/p)
//   k_u_nodeD    D_a = (mu/p) d_a delta Q_a at every node (nodal means)
//   k_u_egrad    again, of D
//   k_u_collide_stream_blk  per block of nodes: F_a = d_a D_a (nodal means)
//                and collision of the block's halo into LDS, then the
//                interpolation below from LDS (k_u_collide + k_u_stream do the
//                same through device memory when a block's halo would not fit)
//   k_u_stream   9-node interpolation at the departure points, which
//                k_u_locate finds once (static mesh) among the node's
//                elements with the corner (first-order) map; then delta Q_a
//                and mu/p of the new populations for the next step
//                (k_u_moments forms them when the host sets populations)
// and, for a moving body, before them: k_u_motion (blended displacements of
// levels n and n+1) and k_u_relocate (the departure points on the mesh of the
// new level, every step).
// A nodal derivative is the mean over the node's elements of the element
// derivative J^{-T} sum_s C_s grad_xi N_s at the node's own local position,
// where only the three nodes on each of the node's element lines contribute
// (the shape functions are Kronecker at the nodes); the element derivatives
// are formed element by element and summed node by node in a fixed order.  Element coordinates are
// FP32 offsets from each element's centre node (formed in FP64 on the host).
// ---------------------------------------------------------------------------
constexpr int U_THREADS = 256;
// departure element of a missing population (block positions)
constexpr uint16_t U_MISSING = 0xffff;
// departure "element" of a rest population whose node does not move: the
// point is the node itself and the population keeps its value (element table
// entry -2; -1 marks a missing population)
constexpr uint16_t U_SELF = 0xfffe;
constexpr int DEP_SELF = -2;

// plane of direction k in the departure tables: the moving directions
// 1..8 in planes 0..7, the rest direction (moving bodies only) in plane 8
__device__ __forceinline__ int dep_plane(int k) { return k == 0 ? 8 : k - 1; }

// Workgroup slot -> block of consecutive nodes (or elements), so that each of
// the 8 XCDs takes a contiguous run of blocks (dispatch slot b goes to XCD
// b mod 8) and the neighbours a block gathers from sit in the same L2.  The
// grid is a multiple of 8; the map is a bijection of [0, gridDim.x).
__device__ __forceinline__ long long xcd_block() {
    const unsigned per = gridDim.x / 8;
    return (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// element node at local position (p, q), p, q in {-1, 0, 1}
__device__ __forceinline__ int q9_node(int p, int q) {
    // rows q = -1, 0, 1; columns p = -1, 0, 1
    const int t[3][3] = {{0, 4, 1}, {7, 8, 5}, {3, 6, 2}};
    return t[q + 1][p + 1];
}
__device__ __forceinline__ int q9_p(int a) { return a == 0 || a == 3 || a == 7 ? -1 : (a == 1 || a == 2 || a == 5 ? 1 : 0); }
__device__ __forceinline__ int q9_q(int a) { return a == 0 || a == 1 || a == 4 ? -1 : (a == 2 || a == 3 || a == 6 ? 1 : 0); }

// derivative at x in {-1, 0, 1} of the quadratic Lagrange basis of node p
__device__ __forceinline__ float dlag_at(int p, int x) {
    if (p < 0) return (float)x - 0.5f;
    if (p == 0) return -2.0f * (float)x;
    return (float)x + 0.5f;
}

// Element pass of a nodal derivative: one thread per element evaluates, at
// each of its nine nodes, d/dx of the first and d/dy of the second component
// of the float2 nodal field `v` (the correction needs only these) and writes
// them to eg[9 e + a].  Differences from the node's own value (the weights of
// each line sum to zero) make the derivative of a constant field exactly zero.
__global__ void __launch_bounds__(U_THREADS) k_u_egrad(const Inst *__restrict__ pinst,
                                                       const float2 *__restrict__ v,
                                                       float2 *__restrict__ eg,
                                                       const double2 *__restrict__ disp) {
    const Inst &P = *pinst;
    for (long long e = xcd_block() * blockDim.x + threadIdx.x; e < P.n_elems;
         e += (long long)gridDim.x * blockDim.x) {
        float2 val[9], rel[9];
#pragma unroll
        for (int s = 0; s < 9; ++s) {
            val[s] = v[P.elems[9 * e + s]];
            rel[s] = P.erel[9 * e + s];
        }
        // the deformed element: offsets from the centre node plus the
        // displacement differences (formed in FP64, rounded once); they are
        // zero where no node moves, and where a translation moves all nodes
        // of a rigid-zone element alike
        const uint8_t ef = disp ? P.eflag[e] : 0;
        if ((ef & Q9E_MOVES) && !((ef & Q9E_RIGID) && !P.q9_rotates)) {
            const double2 dc = disp[P.elems[9 * e + 8]];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const double2 ds = disp[P.elems[9 * e + s]];
                rel[s].x += (float)(ds.x - dc.x);
                rel[s].y += (float)(ds.y - dc.y);
            }
        }
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const int pa = q9_p(a), qa = q9_q(a);
            float axi = 0.0f, aeta = 0.0f, bxi = 0.0f, beta = 0.0f;
            float xxi = 0.0f, yxi = 0.0f, xeta = 0.0f, yeta = 0.0f;
#pragma unroll
            for (int m = -1; m <= 1; ++m) {
                if (m != pa) {
                    const int si = q9_node(m, qa);
                    const float w = dlag_at(m, pa);
                    axi += w * (val[si].x - val[a].x);
                    bxi += w * (val[si].y - val[a].y);
                    xxi += w * (rel[si].x - rel[a].x);
                    yxi += w * (rel[si].y - rel[a].y);
                }
                if (m != qa) {
                    const int sj = q9_node(pa, m);
                    const float w = dlag_at(m, qa);
                    aeta += w * (val[sj].x - val[a].x);
                    beta += w * (val[sj].y - val[a].y);
                    xeta += w * (rel[sj].x - rel[a].x);
                    yeta += w * (rel[sj].y - rel[a].y);
                }
            }
            const float idet = 1.0f / (xxi * yeta - yxi * xeta);
            eg[9 * e + a] = make_float2(idet * (yeta * axi - yxi * aeta), idet * (-xeta * bxi + xxi * beta));
        }
    }
}

// nodal mean of the element derivatives of node idx, summed in the order of
// the node's element list; the first U_PATCH entries are fetched together
// (their loads in flight at once), a longer list continues one by one
constexpr int U_PATCH = 8;
__device__ __forceinline__ float2 node_mean(const Inst &P, const float2 *__restrict__ eg, long long idx) {
    // the first U_PATCH entries from the fixed-stride table (one round trip);
    // a full row may have more: then the CSR lists give the count and the rest
    const int4 pa = reinterpret_cast<const int4 *>(P.patch8)[2 * idx];
    const int4 pb = reinterpret_cast<const int4 *>(P.patch8)[2 * idx + 1];
    const int ent[U_PATCH] = {pa.x, pa.y, pa.z, pa.w, pb.x, pb.y, pb.z, pb.w};
    float2 d[U_PATCH];
#pragma unroll
    for (int j = 0; j < U_PATCH; ++j)
        d[j] = ent[j] >= 0 ? eg[9 * (long long)(ent[j] >> 4) + (ent[j] & 15)] : make_float2(0.0f, 0.0f);
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < U_PATCH; ++j) cnt += ent[j] >= 0 ? 1 : 0;
    float gx = 0.0f, gy = 0.0f;
#pragma unroll
    for (int j = 0; j < U_PATCH; ++j) {
        if (j < cnt) {
            gx += d[j].x;
            gy += d[j].y;
        }
    }
    if (ent[U_PATCH - 1] >= 0) {
        const int b = P.patch_off[idx], e_end = P.patch_off[idx + 1];
        cnt = e_end - b;
        for (int k = b + U_PATCH; k < e_end; ++k) {
            const int e2 = P.patch_ent[k];
            const float2 d2 = eg[9 * (long long)(e2 >> 4) + (e2 & 15)];
            gx += d2.x;
            gy += d2.y;
        }
    }
    const float inv = 1.0f / (float)cnt;
    return make_float2(gx * inv, gy * inv);
}

// delta Q_a and mu/p of a node from its 18 populations, for the correction of
// the step that collides them
__device__ __forceinline__ void u_node_moments(const Inst &P, long long idx, const float f[9],
                                               const float g[9]) {
    const float rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const float jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const float jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const float G = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
    const float ir = 1.0f / rho;
    const float ux = jx * ir, uy = jy * ir;
    const float T = (0.5f * G * ir - 0.5f * (ux * ux + uy * uy)) * (P.gamma - 1.0f);
    const float one3T = 1.0f - 3.0f * T;
    P.uq[idx] = make_float2(jx * (one3T - ux * ux), jy * (one3T - uy * uy));
    P.us[idx] = P.mu / (rho * T);
}

// the moments of the current populations; the interpolation kernels form
// them for the populations they write, so this runs only when the host sets
// the populations (initial state, set, checkpoint load, after a timing pass)
template <int STORE>
__global__ void __launch_bounds__(U_THREADS) k_u_moments(const Inst *__restrict__ pinst) {
    const Inst &P = *pinst;
    const long long n = *P.step;
    const void *src = P.pop[n & 1];
    for (long long idx = xcd_block() * blockDim.x + threadIdx.x; idx < P.n_nodes;
         idx += (long long)gridDim.x * blockDim.x) {
        float f[9], g[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            f[k] = pop_load<STORE>(P, src, k, idx);
            g[k] = pop_load<STORE>(P, src, Q + k, idx);
        }
        u_node_moments(P, idx, f, g);
    }
}

// D_a = (mu / p) d_a delta Q_a at every node
__global__ void __launch_bounds__(U_THREADS) k_u_nodeD(const Inst *__restrict__ pinst) {
    const Inst &P = *pinst;
    for (long long idx = xcd_block() * blockDim.x + threadIdx.x; idx < P.n_nodes;
         idx += (long long)gridDim.x * blockDim.x) {
        const float2 g = node_mean(P, P.ueg, idx);
        const float S = P.us[idx];
        P.ud[idx] = make_float2(S * g.x, S * g.y);
    }
}

template <int STORE>
__global__ void __launch_bounds__(U_THREADS) k_u_collide(const Inst *__restrict__ pinst) {
    const Inst &P = *pinst;
    const long long n = *P.step;
    const void *src = P.pop[n & 1];
    void *dst = P.pop[(n + 1) & 1];
    unsigned err = 0;
    for (long long idx = xcd_block() * blockDim.x + threadIdx.x; idx < P.n_nodes;
         idx += (long long)gridDim.x * blockDim.x) {
        const float2 F = node_mean(P, P.ueg, idx);
        float f[9], g[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            f[k] = pop_load<STORE>(P, src, k, idx);
            g[k] = pop_load<STORE>(P, src, Q + k, idx);
        }
        collide(f, g, F.x, F.y, P, err);
        // rest populations: in place on a fixed mesh; with a moving body after
        // the moving ones (the interpolation moves them where the node moves)
        if (P.qdisp) {
            reinterpret_cast<float2 *>(P.upost)[8 * P.n_nodes + idx] = make_float2(f[0], g[0]);
        } else {
            pop_store<STORE>(P, dst, 0, idx, f[0]);
            pop_store<STORE>(P, dst, Q, idx, g[0]);
        }
        // the 16 moving ones node by node (f_k and g_k of a node side by side,
        // one 64-byte line per node), FP32: the interpolation gathers them
        float4 *up = reinterpret_cast<float4 *>(P.upost) + 4 * idx;
        up[0] = make_float4(f[1], g[1], f[2], g[2]);
        up[1] = make_float4(f[3], g[3], f[4], g[4]);
        up[2] = make_float4(f[5], g[5], f[6], g[6]);
        up[3] = make_float4(f[7], g[7], f[8], g[8]);
    }
    if (err) atomicOr(P.err, err);
}

// Mesh motion of a moving body (Sec. II.D): the blended displacement
// (1 - r)(G'(X) - X) of every node at levels n and n+1 (FP64), for the
// departure points, the deformed elements and the wall.
__global__ void __launch_bounds__(U_THREADS) k_u_motion(const Inst *__restrict__ pinst) {
    const Inst &P = *pinst;
    const long long n = *P.step;
    const BodySlot s0 = P.slots[(n % 3) * MAX_BODIES], s1 = P.slots[((n + 1) % 3) * MAX_BODIES];
    for (long long idx = xcd_block() * blockDim.x + threadIdx.x; idx < P.n_nodes;
         idx += (long long)gridDim.x * blockDim.x) {
        const double2 X = P.X[idx];
        const double om = 1.0 - blend_factor(P, 0, idx, X.x, X.y);
        double d0x, d0y, d1x, d1y;
        rigid_disp(P.body[0], s0, X.x, X.y, d0x, d0y);
        rigid_disp(P.body[0], s1, X.x, X.y, d1x, d1y);
        P.qdisp[idx] = make_double2(om * d0x, om * d0y);
        P.qdisp[P.n_nodes + idx] = make_double2(om * d1x, om * d1y);
    }
}

// Local coordinates of the point at offset (px, py) from local node a of
// element e under the element's corner map (Newton in FP32 from (u, v))
__device__ __forceinline__ void q9_corner_newton(const Inst &P, long long e, int a, float px, float py,
                                                 int iters, float &u, float &v) {
    const float2 *rel = P.erel + 9 * e;
    const float2 c0 = rel[0], c1 = rel[1], c2 = rel[2], c3 = rel[3], ra = rel[a];
    px += ra.x;
    py += ra.y;
    for (int it = 0; it < iters; ++it) {
        const float n0 = (1 - u) * (1 - v), n1 = (1 + u) * (1 - v);
        const float n2 = (1 + u) * (1 + v), n3 = (1 - u) * (1 + v);
        const float rx = 0.25f * (n0 * c0.x + n1 * c1.x + n2 * c2.x + n3 * c3.x) - px;
        const float ry = 0.25f * (n0 * c0.y + n1 * c1.y + n2 * c2.y + n3 * c3.y) - py;
        const float ja = 0.25f * (-(1 - v) * c0.x + (1 - v) * c1.x + (1 + v) * c2.x - (1 + v) * c3.x);
        const float jb = 0.25f * (-(1 - u) * c0.x - (1 + u) * c1.x + (1 + u) * c2.x + (1 - u) * c3.x);
        const float jc = 0.25f * (-(1 - v) * c0.y + (1 - v) * c1.y + (1 + v) * c2.y - (1 + v) * c3.y);
        const float jd = 0.25f * (-(1 - u) * c0.y - (1 + u) * c1.y + (1 + u) * c2.y + (1 - u) * c3.y);
        const float id = 1.0f / (ja * jd - jb * jc);
        u -= id * (jd * rx - jb * ry);
        v -= id * (-jc * rx + ja * ry);
    }
}

// The first element of a node's patch whose corner map holds the point at
// offset (dx, dy) from the node (Newton from the node's own local position);
// e = -1 if none does
__device__ __forceinline__ void u_patch_search(const Inst &P, int b, int e_end, float dx, float dy, int &e,
                                               float &xi, float &eta) {
    for (int q = b; q < e_end && e < 0; ++q) {
        const int ent = P.patch_ent[q], el = ent >> 4, a = ent & 15;
        float u = (float)q9_p(a), v = (float)q9_q(a);
        q9_corner_newton(P, el, a, dx, dy, 8, u, v);
        if (fabsf(u) <= 1.0f + 1e-5f && fabsf(v) <= 1.0f + 1e-5f) {
            e = el;
            xi = u;
            eta = v;
        }
    }
}

// A wall node's departure point, at offset (dx, dy) from the node, located in
// FP64 among the node's elements with their corner (first-order) maps, from
// the FP64 corner coordinates relative to the node: the first element (in
// patch order) that holds it to 1e-12 in local coordinates, else the first
// that holds it to 1e-4 (a point that close to the mesh's boundary counts as
// in the mesh, so that points on the boundary in exact arithmetic, such as the
// rest populations' points of a wall moving along itself, are not decided by
// rounding); e = -1 if none (the population is missing).  Newton from the
// element's centre, stopped once an update falls below 1e-13.
__device__ void q9_wall_locate(const Inst &P, long long idx, double dx, double dy, int &e, float &xi,
                               float &eta) {
    const int b = P.patch_off[idx], cnt = P.patch_off[idx + 1] - b;
    const double2 *cr = P.qw_corner + 4 * (long long)P.qw_coff[P.qw_idx[idx]];
    int e_near = -1;
    double u_near = 0.0, v_near = 0.0;
    e = -1;
    for (int q = 0; q < cnt; ++q) {
        const double2 c0 = cr[4 * q], c1 = cr[4 * q + 1], c2 = cr[4 * q + 2], c3 = cr[4 * q + 3];
        double u = 0.0, v = 0.0;
        bool settled = false;
        for (int it = 0; it < 25; ++it) {
            const double n0 = (1 - u) * (1 - v) * 0.25, n1 = (1 + u) * (1 - v) * 0.25;
            const double n2 = (1 + u) * (1 + v) * 0.25, n3 = (1 - u) * (1 + v) * 0.25;
            const double rx = n0 * c0.x + n1 * c1.x + n2 * c2.x + n3 * c3.x - dx;
            const double ry = n0 * c0.y + n1 * c1.y + n2 * c2.y + n3 * c3.y - dy;
            const double ja = 0.25 * (-(1 - v) * c0.x + (1 - v) * c1.x + (1 + v) * c2.x - (1 + v) * c3.x);
            const double jb = 0.25 * (-(1 - u) * c0.x - (1 + u) * c1.x + (1 + u) * c2.x + (1 - u) * c3.x);
            const double jc = 0.25 * (-(1 - v) * c0.y + (1 - v) * c1.y + (1 + v) * c2.y - (1 + v) * c3.y);
            const double jd = 0.25 * (-(1 - u) * c0.y - (1 + u) * c1.y + (1 + u) * c2.y + (1 - u) * c3.y);
            const double det = ja * jd - jb * jc;
            const double du = (jd * rx - jb * ry) / det, dv = (-jc * rx + ja * ry) / det;
            u -= du;
            v -= dv;
            if (fabs(du) + fabs(dv) < 1e-13) {
                settled = true;
                break;
            }
        }
        if (!settled) continue;
        const double m = fmax(fabs(u), fabs(v));
        if (m <= 1.0 + 1e-12) {
            e = P.patch_ent[b + q] >> 4;
            xi = (float)u;
            eta = (float)v;
            return;
        }
        if (e_near < 0 && m <= 1.0 + 1e-4) {
            e_near = P.patch_ent[b + q] >> 4;
            u_near = u;
            v_near = v;
        }
    }
    if (e_near >= 0) {
        e = e_near;
        xi = (float)u_near;
        eta = (float)v_near;
    }
}

// position of element e (-1: none) in the ascending element list of node
// idx's block (it holds every element of the node's patch)
__device__ __forceinline__ uint16_t u_block_pos(const Inst &P, long long idx, int e) {
    if (e < 0) return e == DEP_SELF ? U_SELF : U_MISSING;
    const long long blk = idx / U_BLOCK;
    int lo = P.be_off[blk], hi = P.be_off[blk + 1];
    const int first = lo;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (P.be_elem[mid] <= e) lo = mid;
        else hi = mid;
    }
    return (uint16_t)(lo - first);
}

// Departure table entry of node idx, direction k: element, local coordinates
// and, with node blocks, the element's position in the block's ascending
// element list (it holds every element of the node's patch); `changed` false
// keeps the element entries (the point stayed in the same element)
__device__ __forceinline__ void u_dep_store(const Inst &P, long long idx, int k, int e, float xi, float eta,
                                            bool changed) {
    const long long at = (long long)dep_plane(k) * P.n_nodes + idx;
    P.dep_xy[at] = make_float2(xi, eta);
    if (!changed) return;
    P.dep_e[at] = e;
    if (P.be_off) P.dep_le[at] = u_block_pos(P, idx, e);
}

// the departure elements' positions in their node blocks' element lists,
// from the element table (after a checkpoint has restored it)
__global__ void __launch_bounds__(U_THREADS) k_u_dep_le(const Inst *__restrict__ pinst) {
    const Inst &P = *pinst;
    const int planes = P.qdisp ? 9 : 8;
    for (long long idx = xcd_block() * blockDim.x + threadIdx.x; idx < P.n_nodes;
         idx += (long long)gridDim.x * blockDim.x)
        for (int k = 0; k < planes; ++k) {
            const long long at = (long long)k * P.n_nodes + idx;
            P.dep_le[at] = u_block_pos(P, idx, P.dep_e[at]);
        }
}

// Departure points of a static mesh, once when the workspace is bound: for
// every node and moving direction the element of the node's patch whose
// corner (first-order) map holds X - dt c_k, and the local coordinates there
// (Newton in FP32 offsets from the element's centre node).  ERR_CFL if an
// interior node's point lies outside every element of its patch; a boundary
// node's point outside them lies outside the mesh: the population is missing
// (set by the boundary kernels).  With a moving body the rest direction's
// entry starts as the node itself (the relocation replaces it where the node
// moves).
__global__ void __launch_bounds__(U_THREADS) k_u_locate(const Inst *__restrict__ pinst) {
    const Inst &P = *pinst;
    const float dt = P.dt;
    unsigned err = 0;
    for (long long idx = xcd_block() * blockDim.x + threadIdx.x; idx < P.n_nodes;
         idx += (long long)gridDim.x * blockDim.x) {
        const int b = P.patch_off[idx], e_end = P.patch_off[idx + 1];
        const bool bnd = P.n_qw + P.n_qf > 0 && (P.qflag[idx] & Q9_BOUNDARY) != 0;
        const bool wallnode = P.n_qw > 0 && (P.qflag[idx] & Q9_WALL) != 0;
        for (int k = 1; k < 9; ++k) {
            int e = -1;
            float xi = 0.0f, eta = 0.0f;
            if (wallnode)
                q9_wall_locate(P, idx, -P.dt_d * (double)CXK(k), -P.dt_d * (double)CYK(k), e, xi, eta);
            else
                u_patch_search(P, b, e_end, -dt * (float)CXK(k), -dt * (float)CYK(k), e, xi, eta);
            if (e < 0 && !bnd) {
                err |= ERR_CFL;
                e = P.patch_ent[b] >> 4;
            }
            u_dep_store(P, idx, k, e, xi, eta, true);
        }
        if (P.qdisp) u_dep_store(P, idx, 0, DEP_SELF, 0.0f, 0.0f, true);
    }
    if (err) atomicOr(P.err, err);
}

// patch entries of a node held in registers by k_u_relocate (larger patches
// take the rest from memory)
constexpr int U_PATCH_REG = 8;

// Departure points of a wall node of a moving body, directions k0 .. k0+nd-1,
// in FP64 (the decision whether a population is missing): g and V_G as in
// u_relocate_dirs, from the FP64 body state and displacements, then
// q9_wall_locate.
__device__ void q9_wall_relocate(const Inst &P, long long idx, int k0, int nd, const BodySlot &s1,
                                 const Body &body) {
    const long long N = P.n_nodes;
    const double2 d0 = P.qdisp[idx], d1 = P.qdisp[N + idx];
    const float2 Lr = P.dgr[3 * idx], LrX = P.dgr[3 * idx + 1], LrY = P.dgr[3 * idx + 2];
    const double A00 = s1.cm1, A01 = -s1.sa, A10 = s1.sa, A11 = s1.cm1;
    const double b0 = -(s1.cm1 * body.ex - s1.sa * body.ey);
    const double b1 = s1.h - (s1.sa * body.ex + s1.cm1 * body.ey);
    const double g00 = 1.0 + A00 - (A00 * LrX.x + A01 * LrY.x) - b0 * Lr.x;
    const double g01 = A01 - (A00 * LrX.y + A01 * LrY.y) - b0 * Lr.y;
    const double g10 = A10 - (A10 * LrX.x + A11 * LrY.x) - b1 * Lr.x;
    const double g11 = 1.0 + A11 - (A10 * LrX.y + A11 * LrY.y) - b1 * Lr.y;
    const double vgx = (d1.x - d0.x) / P.dt_d, vgy = (d1.y - d0.y) / P.dt_d;
    const double det = g00 * g11 - g01 * g10;
    for (int j = 0; j < nd; ++j) {
        const int k = k0 + j;
        if (k == 0 && vgx == 0.0 && vgy == 0.0) {
            u_dep_store(P, idx, 0, DEP_SELF, 0.0f, 0.0f, true);
            continue;
        }
        const double ax = (double)CXK(k) - vgx, ay = (double)CYK(k) - vgy;
        const double dx = -P.dt_d * (g11 * ax - g01 * ay) / det;
        const double dy = -P.dt_d * (-g10 * ax + g00 * ay) / det;
        int e = -1;
        float xi = 0.0f, eta = 0.0f;
        q9_wall_locate(P, idx, dx, dy, e, xi, eta);
        u_dep_store(P, idx, k, e, xi, eta, true);
    }
}

// Departure points of a moving body, every step: X - dt g^{-1}(c_k - V_G) in
// the undeformed frame (k = 0 included: the rest populations' point is
// X + dt g^{-1} V_G, the node itself where V_G = 0), g = I + dd/dX at level n+1 (the nodal mean of the
// element derivatives, formed from the static nodal derivatives of r, r X and
// r Y and the body state), V_G = (d^{n+1} - d^n) / dt; the previous step's
// element is tried first, by Newton from its local coordinates, then the
// patch in order as for a static mesh.  Two threads per node (neighbouring
// lanes, directions 1-4 and 5-8), each issuing its loads in two round trips
// (flag, previous table entries, displacements and the node's first eight
// patch entries at a fixed stride; then the corners of the previous
// elements), rather than one per direction.
constexpr int U_REL_DIRS = 4;   // moving directions per call
template <int ND = U_REL_DIRS>
__device__ __forceinline__ void u_relocate_dirs(const Inst &P, long long idx, int k0, const BodySlot &s1,
                                                const Body &body, unsigned &err) {
    const float dt = P.dt;
    const long long N = P.n_nodes;
    // every load of the node's first round trip, before the flag decides
    // (a patch the blending leaves in place keeps the undeformed mesh's
    // departure points)
    const uint8_t flag = P.qflag[idx];
    const int4 pa = reinterpret_cast<const int4 *>(P.patch8)[2 * idx];
    const int4 pb = reinterpret_cast<const int4 *>(P.patch8)[2 * idx + 1];
    int ep[ND];
    float2 pxy[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        ep[j] = P.dep_e[dep_plane(k0 + j) * N + idx];
        pxy[j] = P.dep_xy[dep_plane(k0 + j) * N + idx];
    }
    const double2 d0 = P.qdisp[idx], d1 = P.qdisp[N + idx];
    const float2 Lr = P.dgr[3 * idx], LrX = P.dgr[3 * idx + 1], LrY = P.dgr[3 * idx + 2];
    if (!(flag & Q9_PATCH_MOVES)) return;
    if (flag & Q9_WALL) {
        q9_wall_relocate(P, idx, k0, ND, s1, body);
        return;
    }
    const bool bnd = (flag & Q9_BOUNDARY) != 0;
    const int ent[U_PATCH_REG] = {pa.x, pa.y, pa.z, pa.w, pb.x, pb.y, pb.z, pb.w};
    // patch size: the entries held, or from the patch offsets for a node
    // with more than eight elements
    int b = 0, e_end = 0, cnt = 0;
#pragma unroll
    for (int j = 0; j < U_PATCH_REG; ++j) cnt += ent[j] >= 0 ? 1 : 0;
    const bool big = ent[U_PATCH_REG - 1] >= 0;
    if (big) {
        b = P.patch_off[idx];
        e_end = P.patch_off[idx + 1];
        cnt = e_end - b;
    }
    // the node's local index in each previous element
    int la[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        la[j] = -1;
#pragma unroll
        for (int i = 0; i < U_PATCH_REG; ++i)
            if (i < cnt && (ent[i] >> 4) == ep[j]) la[j] = ent[i] & 15;
        for (int q = b + U_PATCH_REG; q < e_end; ++q)
            if ((P.patch_ent[q] >> 4) == ep[j]) la[j] = P.patch_ent[q] & 15;
    }
    float2 c0[ND], c1[ND], c2[ND], c3[ND], ra[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        const float2 *rel = P.erel + 9 * (long long)(la[j] >= 0 ? ep[j] : 0);
        c0[j] = rel[0];
        c1[j] = rel[1];
        c2[j] = rel[2];
        c3[j] = rel[3];
        ra[j] = rel[la[j] >= 0 ? la[j] : 0];
    }
    // g = I + A - A L[r X] - b (x) L[r] (the nodal derivative of the
    // displacement (1 - r)(A X + b) of level n+1, A = R(a) - I,
    // b = (0, h) - A X_EA)
    const float A00 = (float)s1.cm1, A01 = (float)(-s1.sa), A10 = (float)s1.sa, A11 = (float)s1.cm1;
    const float b0 = (float)(-(s1.cm1 * body.ex - s1.sa * body.ey));
    const float b1 = (float)(s1.h - (s1.sa * body.ex + s1.cm1 * body.ey));
    const float g00 = 1.0f + A00 - (A00 * LrX.x + A01 * LrY.x) - b0 * Lr.x;
    const float g01 = A01 - (A00 * LrX.y + A01 * LrY.y) - b0 * Lr.y;
    const float g10 = A10 - (A10 * LrX.x + A11 * LrY.x) - b1 * Lr.x;
    const float g11 = 1.0f + A11 - (A10 * LrX.y + A11 * LrY.y) - b1 * Lr.y;
    const float vgx = (float)((d1.x - d0.x) / P.dt_d), vgy = (float)((d1.y - d0.y) / P.dt_d);
    const float idg = 1.0f / (g00 * g11 - g01 * g10);
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        const int k = k0 + j;
        if (k == 0 && vgx == 0.0f && vgy == 0.0f) {
            // a rest population whose node does not move keeps its value
            u_dep_store(P, idx, 0, DEP_SELF, 0.0f, 0.0f, ep[j] != DEP_SELF);
            continue;
        }
        const float ax = (float)CXK(k) - vgx, ay = (float)CYK(k) - vgy;
        const float dx = -dt * idg * (g11 * ax - g01 * ay);
        const float dy = -dt * idg * (-g10 * ax + g00 * ay);
        int e = -1;
        float xi = 0.0f, eta = 0.0f;
        if (la[j] >= 0) {
            // Newton on the previous element's corner map, written as
            // x(u, v) = A + B u + C v + D u v, from the previous local
            // coordinates; the point moves little from step to step, so
            // it stops once an update falls below 1e-6 (at most 4)
            const float2 C0 = c0[j], C1 = c1[j], C2 = c2[j], C3 = c3[j];
            const float Ax = 0.25f * (C0.x + C1.x + C2.x + C3.x) - (dx + ra[j].x);
            const float Ay = 0.25f * (C0.y + C1.y + C2.y + C3.y) - (dy + ra[j].y);
            const float Bx = 0.25f * (-C0.x + C1.x + C2.x - C3.x), By = 0.25f * (-C0.y + C1.y + C2.y - C3.y);
            const float Cx = 0.25f * (-C0.x - C1.x + C2.x + C3.x), Cy = 0.25f * (-C0.y - C1.y + C2.y + C3.y);
            const float Dx = 0.25f * (C0.x - C1.x + C2.x - C3.x), Dy = 0.25f * (C0.y - C1.y + C2.y - C3.y);
            float u = pxy[j].x, v = pxy[j].y;
            for (int it = 0; it < 4; ++it) {
                const float rx = Ax + Bx * u + (Cx + Dx * u) * v;
                const float ry = Ay + By * u + (Cy + Dy * u) * v;
                const float ja = Bx + Dx * v, jb = Cx + Dx * u, jc = By + Dy * v, jd = Cy + Dy * u;
                const float id = 1.0f / (ja * jd - jb * jc);
                const float du = id * (jd * rx - jb * ry), dv = id * (-jc * rx + ja * ry);
                u -= du;
                v -= dv;
                if (fabsf(du) + fabsf(dv) < 1e-6f) break;
            }
            if (fabsf(u) <= 1.0f + 1e-5f && fabsf(v) <= 1.0f + 1e-5f) {
                e = ep[j];
                xi = u;
                eta = v;
            }
        }
        if (e < 0) {
            // left the previous element: the patch in order
            const int pb0 = P.patch_off[idx], pe0 = P.patch_off[idx + 1];
            u_patch_search(P, pb0, pe0, dx, dy, e, xi, eta);
            if (e < 0 && !bnd) {
                err |= ERR_CFL;
                e = P.patch_ent[pb0] >> 4;
            }
        }
        u_dep_store(P, idx, k, e, xi, eta, e != ep[j]);
    }
}

// two threads per node (neighbouring lanes: directions 1-4, and 5-8 then
// the rest direction); the node-block interpolation kernel does the same for
// its own nodes when it runs with the relocation folded in
__global__ void __launch_bounds__(U_THREADS) k_u_relocate(const Inst *__restrict__ pinst) {
    const Inst &P = *pinst;
    const BodySlot s1 = P.slots[((*P.step + 1) % 3) * MAX_BODIES];
    unsigned err = 0;
    for (long long tid = xcd_block() * blockDim.x + threadIdx.x; tid < 2 * P.n_nodes;
         tid += (long long)gridDim.x * blockDim.x) {
        u_relocate_dirs(P, tid >> 1, 1 + U_REL_DIRS * (int)(tid & 1), s1, P.body[0], err);
        if (tid & 1) u_relocate_dirs<1>(P, tid >> 1, 0, s1, P.body[0], err);
    }
    if (err) atomicOr(P.err, err);
}

// 9-node interpolation of the post-collision populations at the tabulated
// departure points, as the node's own value plus weighted differences (the
// weights sum to one), so that constants are reproduced exactly
template <int STORE>
__global__ void __launch_bounds__(U_THREADS) k_u_stream(const Inst *__restrict__ pinst) {
    const Inst &P = *pinst;
    const long long n = *P.step;
    void *dst = P.pop[(n + 1) & 1];
    for (long long idx = xcd_block() * blockDim.x + threadIdx.x; idx < P.n_nodes;
         idx += (long long)gridDim.x * blockDim.x) {
        // the rest populations k_u_collide wrote (fixed mesh), then the moving
        // ones (and with a moving body the rest ones, from after them)
        const bool mv = P.qdisp != nullptr;
        const float2 *up = reinterpret_cast<const float2 *>(P.upost);
        float f[9], g[9];
        if (!mv) {
            f[0] = pop_load<STORE>(P, dst, 0, idx);
            g[0] = pop_load<STORE>(P, dst, Q, idx);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            if (k == 0 && !mv) continue;
            // a missing population (boundary node) is interpolated in element 0
            // at (0, 0), a value the boundary kernels replace
            const int e0 = P.dep_e[dep_plane(k) * P.n_nodes + idx];
            // post-collision (f_k, g_k) of node v
            auto fgk = [&](long long v) { return k == 0 ? up[8 * P.n_nodes + v] : up[8 * v + (k - 1)]; };
            if (e0 == DEP_SELF) {
                const float2 own = fgk(idx);
                pop_store<STORE>(P, dst, k, idx, own.x);
                pop_store<STORE>(P, dst, Q + k, idx, own.y);
                f[k] = pop_round<STORE>(P, k, own.x);
                g[k] = pop_round<STORE>(P, Q + k, own.y);
                continue;
            }
            const int e = e0 < 0 ? 0 : e0;
            const float2 d = P.dep_xy[dep_plane(k) * P.n_nodes + idx];
            const float xi = d.x, eta = d.y;
            const float lx[3] = {0.5f * xi * (xi - 1.0f), 1.0f - xi * xi, 0.5f * xi * (xi + 1.0f)};
            const float ly[3] = {0.5f * eta * (eta - 1.0f), 1.0f - eta * eta, 0.5f * eta * (eta + 1.0f)};
            const int *nodes = P.elems + 9 * (long long)e;
            const float2 fg0 = fgk(idx);
            float vf = fg0.x, vg = fg0.y;
#pragma unroll
            for (int qq = -1; qq <= 1; ++qq)
#pragma unroll
                for (int pp = -1; pp <= 1; ++pp) {
                    const float w = lx[pp + 1] * ly[qq + 1];
                    const float2 fg = fgk(nodes[q9_node(pp, qq)]);
                    vf += w * (fg.x - fg0.x);
                    vg += w * (fg.y - fg0.y);
                }
            pop_store<STORE>(P, dst, k, idx, vf);
            pop_store<STORE>(P, dst, Q + k, idx, vg);
            f[k] = pop_round<STORE>(P, k, vf);
            g[k] = pop_round<STORE>(P, Q + k, vg);
        }
        // moments of the new populations as the next step reads them back
        u_node_moments(P, idx, f, g);
    }
}

// Collision and interpolation of one block of U_BLOCK consecutive nodes, the
// gathers staged through LDS (Morton-ordered meshes keep a block compact): the
// block first collides every node of its halo (the nodes of the elements of
// its nodes; halo nodes are collided by every block that sees them) straight
// into LDS, one plane of (f_k, g_k) per moving direction, and copies the
// block's element lists as halo positions; each node then interpolates from
// LDS.  The same arithmetic as k_u_collide followed by k_u_stream (the
// compiler may fuse multiply-adds differently in the two kernels, so the paths
// agree to FP32 rounding).  Blocks go to XCDs in
// contiguous runs, so neighbouring blocks share their halo's lines in one L2.
//
// With a moving body (MOV) the rest populations form a ninth LDS plane and are
// interpolated like the others where the node moves (a node that does not
// move keeps its own value); on a fixed mesh they go straight to the output.
template <int STORE, int EU16, bool MOV>
__global__ void __launch_bounds__(U_BLOCK) k_u_collide_stream_blk(const Inst *__restrict__ pinst) {
    extern __shared__ __align__(16) unsigned char u_lds[];
    constexpr int NPL = MOV ? 9 : 8;          // LDS planes of (f_k, g_k)
    const Inst &P = *pinst;
    const int nb = P.u_nblk, per_xcd = (nb + 7) / 8;
    const int b = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (b >= nb) return;                              // the whole workgroup
    const long long n = *P.step;
    const void *src = P.pop[n & 1];
    void *dst = P.pop[(n + 1) & 1];
    // the new populations, through a buffer resource: non-temporal where the
    // step streams more than the Infinity Cache holds (a uniform choice; the
    // cache policy is an immediate of each store, so the two stay distinct)
    const bool nt = P.stream_out != 0;
    const PopBuf db = pop_buf<STORE>(P, dst);
    auto store = [&](int q, long long i, float v) {
        const int off = pop_off<STORE>((int)i);
        if (nt)
            pop_st<STORE, true>(P, db, q, off, v);
        else
            pop_st<STORE, false>(P, db, q, off, v);
    };
    const int H = P.u_hmax;
    float2 *pl = reinterpret_cast<float2 *>(u_lds);                                  // [NPL][H]
    uint16_t *el = reinterpret_cast<uint16_t *>(u_lds + (size_t)NPL * H * sizeof(float2));  // [LE][EU16]
    float2 *rest = reinterpret_cast<float2 *>(reinterpret_cast<unsigned char *>(el) +
                                              u_block_elem_bytes(P.u_lemax, EU16));  // [U_BLOCK]
    const int h0 = P.bh_off[b], nh = P.bh_off[b + 1] - h0;
    const int e0 = P.be_off[b], ne = P.be_off[b + 1] - e0;
    const long long n0 = (long long)b * U_BLOCK;
    unsigned err = 0;
    if constexpr (MOV) {
        // a moving body: this block's departure points on the mesh of the new
        // level first (their memory round trips overlap the halo collisions
        // of the other blocks on the CU); the interpolation below reads them
        // back in the same thread
        const long long r = n0 + threadIdx.x;
        if (r < P.n_nodes) {
            const BodySlot s1 = P.slots[((n + 1) % 3) * MAX_BODIES];
            // the rest direction with 1-4, then 5-8: two calls, each with its
            // loads in two memory round trips
            u_relocate_dirs<U_REL_DIRS + 1>(P, r, 0, s1, P.body[0], err);
            u_relocate_dirs(P, r, 1 + U_REL_DIRS, s1, P.body[0], err);
        }
    }
    for (int h = threadIdx.x; h < nh; h += U_BLOCK) {
        const long long v = P.bh_nodes[h0 + h];
        const float2 F = node_mean(P, P.ueg, v);
        float f[9], g[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            f[k] = pop_load<STORE>(P, src, k, v);
            g[k] = pop_load<STORE>(P, src, Q + k, v);
        }
        collide(f, g, F.x, F.y, P, err);
#pragma unroll
        for (int k = 1; k < 9; ++k) pl[(k - 1) * H + h] = make_float2(f[k], g[k]);
        if constexpr (MOV) pl[8 * H + h] = make_float2(f[0], g[0]);
        // fixed mesh, the block's own nodes: rest populations (they do not move)
        const long long own = v - n0;
        if (!MOV && own >= 0 && own < U_BLOCK) {
            store(0, v, f[0]);
            store(Q, v, g[0]);
            rest[own] = make_float2(pop_round<STORE>(P, 0, f[0]), pop_round<STORE>(P, Q, g[0]));
        }
    }
    if (err) atomicOr(P.err, err);
    constexpr int EW = EU16 / 2;            // 32-bit words per element
    const uint32_t *en = reinterpret_cast<const uint32_t *>(P.be_nodes) + EW * (long long)e0;
    uint32_t *elw = reinterpret_cast<uint32_t *>(el);
    for (int x = threadIdx.x; x < EW * ne; x += U_BLOCK) elw[x] = en[x];
    __syncthreads();
    const long long idx = n0 + threadIdx.x;
    if (idx >= P.n_nodes) return;
    const int self = P.uself[idx];
    float f[9], g[9];
    if constexpr (!MOV) {
        f[0] = rest[threadIdx.x].x;
        g[0] = rest[threadIdx.x].y;
    }
#pragma unroll
    for (int k = MOV ? 0 : 1; k < 9; ++k) {
        const float2 *plk = pl + dep_plane(k) * H;
        // a missing population (boundary node) is interpolated in the block's
        // first element at (0, 0), a value the boundary kernels replace
        const int le0 = P.dep_le[dep_plane(k) * P.n_nodes + idx];
        if (k == 0 && le0 == U_SELF) {
            const float2 own = plk[self];
            store(0, idx, own.x);
            store(Q, idx, own.y);
            f[0] = pop_round<STORE>(P, 0, own.x);
            g[0] = pop_round<STORE>(P, Q, own.y);
            continue;
        }
        const int le = le0 == U_MISSING ? 0 : le0;
        const float2 d = P.dep_xy[dep_plane(k) * P.n_nodes + idx];
        const float xi = d.x, eta = d.y;
        const float lx[3] = {0.5f * xi * (xi - 1.0f), 1.0f - xi * xi, 0.5f * xi * (xi + 1.0f)};
        const float ly[3] = {0.5f * eta * (eta - 1.0f), 1.0f - eta * eta, 0.5f * eta * (eta + 1.0f)};
        const uint32_t *ew = elw + EW * le;
        uint32_t w0, w1, w2, w3;
        if constexpr (EU16 == 16) {
            const uint4 v = *reinterpret_cast<const uint4 *>(ew);
            w0 = v.x; w1 = v.y; w2 = v.z; w3 = v.w;
        } else if constexpr (EU16 == 12) {
            const uint2 v0 = *reinterpret_cast<const uint2 *>(ew);
            const uint2 v1 = *reinterpret_cast<const uint2 *>(ew + 2);
            w0 = v0.x; w1 = v0.y; w2 = v1.x; w3 = v1.y;
        } else {
            w0 = ew[0]; w1 = ew[1]; w2 = ew[2]; w3 = ew[3];
        }
        const int n8 = (int)(ew[4] & 0xffffu);
        const int nodes[9] = {(int)(w0 & 0xffffu), (int)(w0 >> 16), (int)(w1 & 0xffffu),
                              (int)(w1 >> 16),     (int)(w2 & 0xffffu), (int)(w2 >> 16),
                              (int)(w3 & 0xffffu), (int)(w3 >> 16),     n8};
        const float2 fg0 = plk[self];
        float vf = fg0.x, vg = fg0.y;
#pragma unroll
        for (int qq = -1; qq <= 1; ++qq)
#pragma unroll
            for (int pp = -1; pp <= 1; ++pp) {
                const float w = lx[pp + 1] * ly[qq + 1];
                const float2 fg = plk[nodes[q9_node(pp, qq)]];
                vf += w * (fg.x - fg0.x);
                vg += w * (fg.y - fg0.y);
            }
        store(k, idx, vf);
        store(Q + k, idx, vg);
        f[k] = pop_round<STORE>(P, k, vf);
        g[k] = pop_round<STORE>(P, Q + k, vg);
    }
    u_node_moments(P, idx, f, g);
}

// ---------------------------------------------------------------------------
// Boundary of a bounded Q9 mesh round a fixed body (Sec. III.A, III):
//   k_u_far           far-field nodes: free-stream equilibrium
//   k_u_wall_targets  rho, T at B (9-node interpolation in the element that
//                     holds B; wall nodes there at their previous values)
//   k_u_wall          Grad populations for the missing ones (gradients by the
//                     nodal finite-element derivative, wall nodes at their
//                     targets), moments for the next step, traction, and the
//                     wall node's (rho, T) for the next step's targets
// One thread per far-field node, one wave per wall node; run after the
// interpolation.
// ---------------------------------------------------------------------------
constexpr int U_BND = 64;

template <int STORE>
__global__ void __launch_bounds__(U_BND) k_u_far(const Inst *__restrict__ pinst) {
    const Inst &P = *pinst;
    const int k = blockIdx.x * U_BND + threadIdx.x;
    if (k >= P.n_qf) return;
    const long long n = *P.step;
    void *dst = P.pop[(n + 1) & 1];
    const long long v = P.qf_nodes[k];
    const float T = P.T_inf, ux = P.ux_inf, uy = P.uy_inf;
    const float E = P.Cv * T + 0.5f * (ux * ux + uy * uy);
    float f[9], g[9];
    equilibria<float>(P.rho_inf, ux, uy, T, E, f, g);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        pop_store<STORE>(P, dst, q, v, f[q]);
        pop_store<STORE>(P, dst, Q + q, v, g[q]);
        f[q] = pop_round<STORE>(P, q, f[q]);
        g[q] = pop_round<STORE>(P, Q + q, g[q]);
    }
    u_node_moments(P, v, f, g);
}

// one wave per wall node: nine lanes fetch the element's node values at once
template <int STORE>
__global__ void __launch_bounds__(64) k_u_wall_targets(const Inst *__restrict__ pinst) {
    __shared__ float sv[9][2];
    const Inst &P = *pinst;
    const int k = blockIdx.x, t = threadIdx.x;
    if (k >= P.n_qw) return;
    const long long n = *P.step;
    const void *dst = P.pop[(n + 1) & 1];
    const int e = P.qw_eB[k];
    if (t < 9) {
        const long long v = P.elems[9 * (long long)e + t];
        const int wi = P.qw_idx[v];
        float r, T;
        if (wi >= 0) {
            const float2 pv = P.qw_prev[wi];
            r = pv.x;
            T = pv.y;
        } else {
            float f[9], g[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                f[q] = pop_load<STORE>(P, dst, q, v);
                g[q] = pop_load<STORE>(P, dst, Q + q, v);
            }
            const Moments m = moments(f, g, P.Cv);
            r = m.rho;
            T = m.T;
        }
        sv[t][0] = r;
        sv[t][1] = T;
    }
    __syncthreads();
    if (t != 0) return;
    const float2 B = P.qw_xyB[k];
    const float lx[3] = {0.5f * B.x * (B.x - 1.0f), 1.0f - B.x * B.x, 0.5f * B.x * (B.x + 1.0f)};
    const float ly[3] = {0.5f * B.y * (B.y - 1.0f), 1.0f - B.y * B.y, 0.5f * B.y * (B.y + 1.0f)};
    float rho_t = 0.0f, T_t = 0.0f;
    for (int s2 = 0; s2 < 9; ++s2) {
        const float w = lx[q9_p(s2) + 1] * ly[q9_q(s2) + 1];
        rho_t += w * sv[s2][0];
        T_t += w * sv[s2][1];
    }
    P.wall_tgt[k] = make_float4(rho_t, 0.0f, 0.0f, T_t);
}

// mesh velocity V_G = (d^{n+1} - d^n) / dt of node v (moving body)
__device__ __forceinline__ float2 q9_mesh_velocity(const Inst &P, long long v) {
    const double2 d0 = P.qdisp[v], d1 = P.qdisp[P.n_nodes + v];
    return make_float2((float)((d1.x - d0.x) / P.dt_d), (float)((d1.y - d0.y) / P.dt_d));
}

// (u_x, u_y, T, E) of node v for a wall node's gradient: the target at wall
// nodes (the wall's mesh velocity, zero for a fixed body), the moments of the
// new populations elsewhere
template <int STORE>
__device__ float4 q9_wall_field(const Inst &P, const void *buf, long long v) {
    const int wi = P.qw_idx[v];
    if (wi >= 0) {
        const float T = P.wall_tgt[wi].w;
        const float2 u = P.qdisp ? q9_mesh_velocity(P, v) : make_float2(0.0f, 0.0f);
        return make_float4(u.x, u.y, T, P.Cv * T + 0.5f * (u.x * u.x + u.y * u.y));
    }
    float f[9], g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        f[q] = pop_load<STORE>(P, buf, q, v);
        g[q] = pop_load<STORE>(P, buf, Q + q, v);
    }
    const Moments m = moments(f, g, P.Cv);
    return make_float4(m.ux, m.uy, m.T, m.E);
}

// element lines through local node a: the two other nodes along xi (r = 0, 1)
// and along eta (r = 2, 3), with their derivative weights at a
__device__ __forceinline__ void wall_line_node(int a, int r, int &s, float &w) {
    const int pa = q9_p(a), qa = q9_q(a);
    int cnt = 0;
    s = a;
    w = 0.0f;
    for (int m = -1; m <= 1; ++m) {
        if (r < 2 && m != pa && cnt++ == r) { s = q9_node(m, qa); w = dlag_at(m, pa); }
        if (r >= 2 && m != qa && cnt++ == r - 2) { s = q9_node(pa, m); w = dlag_at(m, qa); }
    }
}

// one wave per wall node: lanes fetch the line nodes of the node's elements
// at once (four per element), the element derivatives follow per element, and
// one lane completes the node
constexpr int U_WALL_ENT = 16;   // elements of a wall node handled per pass
template <int STORE>
__global__ void __launch_bounds__(64) k_u_wall(const Inst *__restrict__ pinst, int phase) {
    __shared__ float4 sval[U_WALL_ENT][4];
    __shared__ float sder[U_WALL_ENT][4][2];
    __shared__ float sgrad[4][2];
    const Inst &P = *pinst;
    const int k = blockIdx.x, t = threadIdx.x;
    if (k >= P.n_qw) return;
    const long long n = *P.step;
    void *buf = P.pop[(phase ? n + 1 : n) & 1];
    const long long w = P.qw_nodes[k];
    const bool mv = P.qdisp != nullptr;
    // missing populations: departure point outside the mesh (the rest
    // populations only with a moving body)
    unsigned miss = 0;
    for (int q = mv ? 0 : 1; q < 9; ++q)
        if (P.dep_e[dep_plane(q) * P.n_nodes + w] == -1) miss |= 1u << q;
    const float4 t0 = P.wall_tgt[k];
    // the wall's mesh velocity (no slip), the displacements of the level
    const float2 uw = mv && phase ? q9_mesh_velocity(P, w) : make_float2(0.0f, 0.0f);
    const double2 *dL = mv ? P.qdisp + (phase ? P.n_nodes : 0) : nullptr;
    const float T_t = t0.w, E_t = P.Cv * T_t + 0.5f * (uw.x * uw.x + uw.y * uw.y);
    const bool fill = phase && miss;
    if (fill) {
        // nodal derivative: mean over the node's elements of the element
        // derivative at the node (the nodes on its two element lines), the
        // wall nodes at their targets
        const int b = P.patch_off[w], e_end = P.patch_off[w + 1];
        const float4 Ca = make_float4(uw.x, uw.y, T_t, E_t);
        float acc[4][2] = {};
        for (int base = b; base < e_end; base += U_WALL_ENT) {
            const int cnt = min(U_WALL_ENT, e_end - base);
            if (t < 4 * cnt) {
                const int j = t >> 2, r = t & 3;
                const int ent = P.patch_ent[base + j], e = ent >> 4, a = ent & 15;
                int sn;
                float wt;
                wall_line_node(a, r, sn, wt);
                sval[j][r] = q9_wall_field<STORE>(P, buf, P.elems[9 * (long long)e + sn]);
            }
            __syncthreads();
            if (t < cnt) {
                const int ent = P.patch_ent[base + t], e = ent >> 4, a = ent & 15;
                const float2 *rel = P.erel + 9 * (long long)e;
                float ax[4] = {}, ae[4] = {};
                float xxi = 0.0f, yxi = 0.0f, xeta = 0.0f, yeta = 0.0f;
                for (int r = 0; r < 4; ++r) {
                    int sn;
                    float wt;
                    wall_line_node(a, r, sn, wt);
                    const float4 C = sval[t][r];
                    const float dC[4] = {C.x - Ca.x, C.y - Ca.y, C.z - Ca.z, C.w - Ca.w};
                    float dx = rel[sn].x - rel[a].x, dy = rel[sn].y - rel[a].y;
                    if (mv) {                 // the deformed element of the new level
                        const double2 ds = dL[P.elems[9 * (long long)e + sn]], da = dL[P.elems[9 * (long long)e + a]];
                        dx += (float)(ds.x - da.x);
                        dy += (float)(ds.y - da.y);
                    }
                    if (r < 2) {
                        for (int c = 0; c < 4; ++c) ax[c] += wt * dC[c];
                        xxi += wt * dx;
                        yxi += wt * dy;
                    } else {
                        for (int c = 0; c < 4; ++c) ae[c] += wt * dC[c];
                        xeta += wt * dx;
                        yeta += wt * dy;
                    }
                }
                const float idet = 1.0f / (xxi * yeta - yxi * xeta);
                for (int c = 0; c < 4; ++c) {
                    sder[t][c][0] = idet * (yeta * ax[c] - yxi * ae[c]);
                    sder[t][c][1] = idet * (-xeta * ax[c] + xxi * ae[c]);
                }
            }
            __syncthreads();
            if (t == 0)
                for (int j = 0; j < cnt; ++j)
                    for (int c = 0; c < 4; ++c) {
                        acc[c][0] += sder[j][c][0];
                        acc[c][1] += sder[j][c][1];
                    }
            __syncthreads();
        }
        if (t == 0) {
            const float inv = 1.0f / (float)(e_end - b);
            for (int c = 0; c < 4; ++c) {
                sgrad[c][0] = acc[c][0] * inv;
                sgrad[c][1] = acc[c][1] * inv;
            }
        }
    }
    if (t != 0) return;
    float f[9], g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        f[q] = pop_load<STORE>(P, buf, q, w);
        g[q] = pop_load<STORE>(P, buf, Q + q, w);
    }
    if (fill) {
        grad_populations(P, miss, t0.x, uw.x, uw.y, T_t, E_t, sgrad[0][0], sgrad[0][1], sgrad[1][0],
                         sgrad[1][1], sgrad[2][0], sgrad[2][1], sgrad[3][0], sgrad[3][1], f, g);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            if (!(miss & (1u << q))) continue;
            pop_store<STORE>(P, buf, q, w, f[q]);
            pop_store<STORE>(P, buf, Q + q, w, g[q]);
            f[q] = pop_round<STORE>(P, q, f[q]);
            g[q] = pop_round<STORE>(P, Q + q, g[q]);
        }
    }
    if (phase) u_node_moments(P, w, f, g);
    // traction of the complete wall node; its (rho, T) for the next targets
    double sxx, sxy, syy;
    const bool ok = wall_stress(P, f, g, sxx, sxy, syy);
    double4 geo = P.qw_geo[k];
    if (mv) {
        // lumped normal and moment arm on the mesh of the level
        const int nw = P.n_qw;
        const long long vm = P.qw_nodes[(k + nw - 1) % nw], vp = P.qw_nodes[(k + 1) % nw];
        const double2 Xm = P.X[vm], Xp = P.X[vp], Xw = P.X[w];
        const double2 dm = dL[vm], dp = dL[vp], dw = dL[w];
        const double h = P.slots[((phase ? n + 1 : n) % 3) * MAX_BODIES].h;
        geo = make_double4(-0.5 * ((Xp.y + dp.y) - (Xm.y + dm.y)), 0.5 * ((Xp.x + dp.x) - (Xm.x + dm.x)),
                           Xw.x + dw.x - P.body[0].ex, Xw.y + dw.y - (P.body[0].ey + h));
    }
    const double Fx = sxx * geo.x + sxy * geo.y;
    const double Fy = sxy * geo.x + syy * geo.y;
    P.wall_force[k] = make_double4(Fx, Fy, geo.z * Fy - geo.w * Fx, 0.0);
    const Moments m = moments(f, g, P.Cv);
    P.qw_prev[k] = make_float2(m.rho, m.T);
    if (!ok) atomicOr(P.err, ERR_STATE);
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
hipError_t launch_unstructured_locate(const Inst *inst, long long n_nodes, hipStream_t s) {
    const long long g64 = ((n_nodes + 8 * U_THREADS - 1) / (8 * U_THREADS)) * 8;
    hipLaunchKernelGGL(k_u_locate, dim3((unsigned)(g64 > 0 ? g64 : 8)), dim3(U_THREADS), 0, s, inst);
    return hipGetLastError();
}

hipError_t launch_unstructured_dep_le(const Inst *inst, long long n_nodes, hipStream_t s) {
    const long long g64 = ((n_nodes + 8 * U_THREADS - 1) / (8 * U_THREADS)) * 8;
    hipLaunchKernelGGL(k_u_dep_le, dim3((unsigned)(g64 > 0 ? g64 : 8)), dim3(U_THREADS), 0, s, inst);
    return hipGetLastError();
}

hipError_t launch_unstructured_moments(const Inst *inst, long long n_nodes, int storage, hipStream_t s) {
    const long long g64 = ((n_nodes + 8 * U_THREADS - 1) / (8 * U_THREADS)) * 8;
    FSI_DISPATCH(storage, k_u_moments, dim3((unsigned)(g64 > 0 ? g64 : 8)), dim3(U_THREADS), s, inst);
    return hipGetLastError();
}

hipError_t launch_unstructured(const Inst *inst, long long n_nodes, long long n_elems, int storage,
                               float2 *uq, float2 *ud, float2 *ueg, int n_blocks, int hmax, int lemax,
                               int eu16, const double2 *disp0, int relocate, hipStream_t s) {
    // multiples of the XCD count (see xcd_block)
    const long long g64 = ((n_nodes + 8 * U_THREADS - 1) / (8 * U_THREADS)) * 8;
    const long long e64 = ((n_elems + 8 * U_THREADS - 1) / (8 * U_THREADS)) * 8;
    const dim3 grid((unsigned)(g64 > 0 ? g64 : 8)), egrid((unsigned)(e64 > 0 ? e64 : 8)), block(U_THREADS);
    hipLaunchKernelGGL(k_u_egrad, egrid, block, 0, s, inst, uq, ueg, disp0);
    hipLaunchKernelGGL(k_u_nodeD, grid, block, 0, s, inst);
    hipLaunchKernelGGL(k_u_egrad, egrid, block, 0, s, inst, ud, ueg, disp0);
    if (n_blocks > 0) {
        // a multiple of the XCD count; the kernel maps slots to blocks
        const unsigned g = (unsigned)(((n_blocks + 7) / 8) * 8);
        const size_t lds = u_block_lds_bytes(hmax, lemax, eu16, relocate ? 9 : 8);
#define FSI_U_BLK(ST, EU)                                                                          \
    do {                                                                                           \
        if (relocate)                                                                              \
            hipLaunchKernelGGL((k_u_collide_stream_blk<ST, EU, true>), dim3(g), dim3(U_BLOCK), lds, s, inst); \
        else                                                                                       \
            hipLaunchKernelGGL((k_u_collide_stream_blk<ST, EU, false>), dim3(g), dim3(U_BLOCK), lds, s, inst); \
    } while (0)
        if (storage == 0) {
            if (eu16 == 16) FSI_U_BLK(0, 16);
            else if (eu16 == 12) FSI_U_BLK(0, 12);
            else FSI_U_BLK(0, 10);
        } else {
            if (eu16 == 16) FSI_U_BLK(1, 16);
            else if (eu16 == 12) FSI_U_BLK(1, 12);
            else FSI_U_BLK(1, 10);
        }
#undef FSI_U_BLK
    } else {
        FSI_DISPATCH(storage, k_u_collide, grid, block, s, inst);
        FSI_DISPATCH(storage, k_u_stream, grid, block, s, inst);
    }
    return hipGetLastError();
}

hipError_t launch_unstructured_motion(const Inst *inst, long long n_nodes, long long n_elems, int relocate,
                                      hipStream_t s) {
    const long long g64 = ((n_nodes + 8 * U_THREADS - 1) / (8 * U_THREADS)) * 8;
    hipLaunchKernelGGL(k_u_motion, dim3((unsigned)g64), dim3(U_THREADS), 0, s, inst);
    if (relocate) {
        // two threads per node
        const long long r64 = ((2 * n_nodes + 8 * U_THREADS - 1) / (8 * U_THREADS)) * 8;
        hipLaunchKernelGGL(k_u_relocate, dim3((unsigned)r64), dim3(U_THREADS), 0, s, inst);
    }
    return hipGetLastError();
}

hipError_t launch_unstructured_boundary(const Inst *inst, int n_wall, int n_far, int storage, int phase,
                                        hipStream_t s) {
    const dim3 block(U_BND);
    if (phase && n_far > 0)
        FSI_DISPATCH(storage, k_u_far, dim3((n_far + U_BND - 1) / U_BND), block, s, inst);
    if (n_wall > 0) {
        // one wave per wall node
        if (phase) FSI_DISPATCH(storage, k_u_wall_targets, dim3(n_wall), dim3(64), s, inst);
        FSI_DISPATCH(storage, k_u_wall, dim3(n_wall), dim3(64), s, inst, phase);
    }
    return hipGetLastError();
}

}  // namespace fsi
