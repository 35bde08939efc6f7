// Host runtime of the C ABI declared in include/fsilbm.h: validation, static
// boundary geometry, workspace layout, graph capture of one coupled step, and
// host <-> device transfers.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/fsilbm.h"
#include "fsilbm_internal.h"

using fsi::Inst;

// Per-step scratch of fsi_step_noalloc (callers that cannot allocate): the
// wall masks, wall targets, per-node tractions and cut staging of one step,
// which fsi_step keeps in the caller's workspace.  One copy per GPU, held
// until the process ends; every call on a GPU shares it, so calls that
// overlap on one GPU race.  Host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (noalloc_scratch below).
constexpr size_t kNoAllocScratchBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

struct fsi_ctx {
    fsi_fluid_params fluid{};
    int ni = 0, nj = 0, topo = 0, n_wake = 0, n_wall2 = 0;
    bool has_wall = false;      // O-grid, C-grid or twin O-grid
    bool cut = false;           // C-grid or twin O-grid
    int shape = 0;              // work-item shape of the fused kernel (fsi::TILE_SHAPES)
    bool stream_out = false;    // the step streams more than the Infinity Cache holds
    int cut_a = 0, cut_b = 0, mirror = 0;
    int seg_i0[fsi::MAX_BODIES] = {}, seg_n[fsi::MAX_BODIES] = {}, seg_dup[fsi::MAX_BODIES] = {};
    int n_seg = 0;
    double shift_i[2] = {0, 0}, shift_j[2] = {0, 0};
    std::vector<double> X;          // [nj][ni][2]
    std::vector<fsi_body_desc> bodies;
    // unstructured 9-node meshes
    int n_elems = 0;
    std::vector<int> elems;         // [E][9]
    std::vector<float2> erel;       // [E][9] offsets from the element's centre node
    std::vector<int> patch_off, patch_ent;
    std::vector<int> patch8;            // [N][8] first patch entries, -1 past the end
    std::vector<float2> q9_dgr;         // moving body: [N][3] nodal derivatives of r, r X, r Y
    std::vector<uint8_t> q9_eflag;      // moving body: [E] Q9E_MOVES, Q9E_RIGID
    // node blocks of the LDS-staged interpolation (empty: device-memory gathers)
    std::vector<int> bh_off, bh_nodes, be_off, be_elem;
    std::vector<uint16_t> be_nodes, uself;
    int u_hmax = 0, u_lemax = 0, u_eu16 = 16;
    // unstructured meshes round a fixed body
    std::vector<uint8_t> qflag;
    std::vector<int> qw_nodes, qw_idx, qf_nodes, qw_eB;
    std::vector<double4> qw_geo;
    std::vector<float2> qw_xyB;
    // per wall node: the corners of its elements (patch order) relative to the
    // node in FP64, for the wall nodes' FP64 departure-point location
    std::vector<int> qw_coff;       // [n_qw + 1] first patch entry of each wall node
    std::vector<double2> qw_corner; // [entries][4]
    std::vector<double> ecoord;     // [E][9][2] unwrapped FP64 element node coordinates
    bool q9_moving = false;         // a moving body on a Q9 mesh
    hipStream_t stream = nullptr;
    // O-grids: wk1s holds the fused kernel's tiles with a row the boundary
    // kernels read or write (rows 0..2, nj-2, nj-1) first (n_near of them),
    // then the others, which do not depend on the boundary kernels of their
    // step: on a large instance fsi_step runs them on a second stream beside
    // the near tiles and the boundary kernels, joining before the body kernel
    // (which advances the step).  wk1 keeps every tile in one list for single
    // launches.
    std::vector<int2> wk1s;
    size_t off_wk1s = 0;
    int n_near = 0;
    bool split = false;
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int n_sub = 1;                  // coupling sub-iterations per step
    double relax = 1.0;
    Inst inst{};
    // workspace layout (byte offsets)
    size_t off_pop[2]{}, off_X = 0, off_mask = 0, off_tgt = 0, off_B = 0, off_inflow = 0,
           off_force = 0, off_slots = 0, off_hist = 0, off_step = 0, off_err = 0, off_inst = 0,
           off_wk1 = 0, off_wbnd = 0, off_wwall = 0, off_ff = 0, off_cut = 0, off_wk0 = 0, off_dist = 0,
           off_resid = 0, off_elems = 0, off_erel = 0, off_poff = 0, off_pent = 0, off_uq = 0,
           off_ud = 0, off_upost = 0, off_dep_e = 0, off_dep_xy = 0, off_us = 0, off_ueg = 0,
           off_bh_off = 0, off_bh_nodes = 0, off_be_off = 0, off_be_elem = 0, off_be_nodes = 0,
           off_uself = 0, off_dep_le = 0, off_qflag = 0, off_qw = 0, off_qwidx = 0, off_qf = 0,
           off_qwgeo = 0, off_qweB = 0, off_qwxyB = 0, off_qwprev = 0, off_qdisp = 0, off_dgr = 0, off_eflag = 0, off_patch8 = 0,
           off_qwcoff = 0, off_qwcorner = 0,
           total = 0;
    char *ws = nullptr;
    std::vector<float2> wallB;
    std::vector<double> wall_dist;      // blend_mode 1: [body][node] distance to the body's wall
    std::vector<uint8_t> inflow;        // per far-field list entry
    std::vector<int2> ff;               // far-field (node, interior node)
    std::vector<int2> wk0, wk1, wbnd, wwall;
    // fsi_step_noalloc: a second device copy of the instance whose per-step
    // scratch pointers lead into the static scratch array of the bound device
    size_t off_inst_na = 0;
    size_t na_bytes = 0;            // scratch the step needs (0: not supported)
    bool na_ready = false;          // the copy is uploaded
    // captured steps: [0] one step, [1] kGraphSteps steps (fewer graph launches)
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    int64_t host_step = 0;
    bool initialized = false;
    std::string err;
};

namespace {

constexpr int64_t kMagic = 0x46534c424d303032LL;   // checkpoint tag

fsi_status fail(fsi_ctx *c, fsi_status st, const std::string &msg) {
    if (c) c->err = msg;
    return st;
}

fsi_status hip_fail(fsi_ctx *c, hipError_t e, const char *what) {
    return fail(c, FSI_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(c, expr)                                   \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_fail(c, e_, #expr); \
    } while (0)

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Device address of the static scratch array on the current device, looked up
// once per device (each GPU holds its own copy at its own address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

hipError_t noalloc_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// byte offsets of the per-step scratch inside the static array: wall masks
// (missing, ambiguous), wall targets, tractions, cut staging; the total
size_t na_layout(const fsi_ctx *c, size_t off[5]) {
    size_t o = 0;
    const size_t sz[5] = {(size_t)c->ni * 4, (size_t)c->ni * 16, (size_t)c->ni * 32,
                          (size_t)18 * c->inst.cut_n * sizeof(float), 0};
    for (int k = 0; k < 5; ++k) {
        off[k] = o;
        o += align_up(sz[k]);
    }
    return o;
}

int wrapi(int a, int n) { return ((a % n) + n) % n; }

// coordinate of node (i, j) seen from an unwrapped index, with periodic shifts
void coord(const fsi_ctx *c, int i, int j, double &x, double &y) {
    if (c->cut) {
        if (j < 0) {                       // across the cut
            i = c->mirror - i;
            j = -j;
        }
        if (c->topo == FSI_TOPO_TWIN) i = wrapi(i, c->ni);
        x = c->X[2 * ((size_t)j * c->ni + i)];
        y = c->X[2 * ((size_t)j * c->ni + i) + 1];
        return;
    }
    const int wi = (int)floor((double)i / c->ni), wj = (int)floor((double)j / c->nj);
    const int ii = i - wi * c->ni;
    const int jj = c->topo == FSI_TOPO_PERIODIC2 ? j - wj * c->nj : j;
    x = c->X[2 * ((size_t)jj * c->ni + ii)];
    y = c->X[2 * ((size_t)jj * c->ni + ii) + 1];
    x += wi * c->shift_i[0];
    y += wi * c->shift_i[1];
    if (c->topo == FSI_TOPO_PERIODIC2) {
        x += wj * c->shift_j[0];
        y += wj * c->shift_j[1];
    }
}

// bilinear inverse of cell with corners (relative) c00, c10, c01, c11 -> (s, t)
bool bilinear_inverse(const double c[4][2], double px, double py, double &s, double &t) {
    s = 0.5;
    t = 0.5;
    for (int it = 0; it < 60; ++it) {
        const double ax = c[1][0] - c[0][0], ay = c[1][1] - c[0][1];
        const double bx = c[2][0] - c[0][0], by = c[2][1] - c[0][1];
        const double ex = c[3][0] - c[1][0] - c[2][0] + c[0][0], ey = c[3][1] - c[1][1] - c[2][1] + c[0][1];
        const double rx = c[0][0] + ax * s + bx * t + ex * s * t - px;
        const double ry = c[0][1] + ay * s + by * t + ey * s * t - py;
        const double jsx = ax + ex * t, jsy = ay + ey * t, jtx = bx + ex * s, jty = by + ey * s;
        const double det = jsx * jty - jsy * jtx;
        if (!(fabs(det) > 0)) return false;
        const double ds = (jty * rx - jtx * ry) / det, dt = (-jsy * rx + jsx * ry) / det;
        s -= ds;
        t -= dt;
        if (fabs(ds) + fabs(dt) < 1e-15) break;
    }
    return isfinite(s) && isfinite(t);
}

// blending factor of body b at (X, Y), d_wall its distance to the body's wall
// (distance blending)
double blend_r(const fsi_body_desc &b, double X, double Y, double d_wall = 0.0) {
    const double d = b.blend_mode == 1 ? d_wall : hypot(X - b.center[0], Y - b.center[1]);
    const double s = (d - b.r_rigid) / (b.r_blend - b.r_rigid);
    if (s <= 0) return 0;
    if (s >= 1) return 1;
    return s * s * s * (10 + s * (-15 + 6 * s));
}

fsi::BodySlot slot_of(double h, double a, double hd, double ad) {
    fsi::BodySlot s{};
    s.h = h; s.a = a; s.hd = hd; s.ad = ad;
    const double sh = sin(0.5 * a);
    s.cm1 = -2.0 * sh * sh;
    s.sa = sin(a);
    return s;
}

int mirror_of(const fsi_ctx *c, int i) {
    const int m = c->mirror - i;
    return c->topo == FSI_TOPO_TWIN ? wrapi(m, c->ni) : m;
}

bool is_cut_col(const fsi_ctx *c, int i) {
    if (!c->cut) return false;
    const int m = mirror_of(c, i);
    return (i > c->cut_a && i < c->cut_b) || (m > c->cut_a && m < c->cut_b);
}

bool is_wall_col(const fsi_ctx *c, int i) { return c->has_wall && !is_cut_col(c, i); }

// index-space FE derivative of the undeformed coordinates at node (i, j):
// centred, one-sided 3-point on wall columns of row 0, on row nj - 1 and on
// the exit columns of a C-grid; across the cut (mirror) on C-grid cut columns
void dX_di(const fsi_ctx *c, int i, int j, double &xd, double &yd) {
    double x0, y0, x1, y1, x2, y2;
    if (c->topo == FSI_TOPO_CGRID && (i == 0 || i == c->ni - 1)) {
        const int s = i == 0 ? 1 : -1;
        coord(c, i, j, x0, y0);
        coord(c, i + s, j, x1, y1);
        coord(c, i + 2 * s, j, x2, y2);
        xd = s * (2.0 * (x1 - x0) - 0.5 * (x2 - x0));
        yd = s * (2.0 * (y1 - y0) - 0.5 * (y2 - y0));
        return;
    }
    coord(c, i + 1, j, x1, y1);
    coord(c, i - 1, j, x0, y0);
    xd = 0.5 * (x1 - x0);
    yd = 0.5 * (y1 - y0);
}

void dX_dj(const fsi_ctx *c, int i, int j, double &xd, double &yd) {
    double x0, y0, x1, y1, x2, y2;
    const bool wall_row = c->has_wall && j == 0 && is_wall_col(c, i);
    if (wall_row || (c->has_wall && j == c->nj - 1)) {
        const int s = j == 0 ? 1 : -1;
        coord(c, i, j, x0, y0);
        coord(c, i, j + s, x1, y1);
        coord(c, i, j + 2 * s, x2, y2);
        xd = s * (2.0 * (x1 - x0) - 0.5 * (x2 - x0));
        yd = s * (2.0 * (y1 - y0) - 0.5 * (y2 - y0));
        return;
    }
    coord(c, i, j + 1, x1, y1);
    coord(c, i, j - 1, x0, y0);
    xd = 0.5 * (x1 - x0);
    yd = 0.5 * (y1 - y0);
}

// cut constants and wall segments of the topology (sizes validated first)
fsi_status topology(fsi_ctx *c) {
    const int ni = c->ni;
    c->cut = c->topo == FSI_TOPO_CGRID || c->topo == FSI_TOPO_TWIN;
    c->n_seg = 0;
    if (c->topo == FSI_TOPO_OGRID) {
        c->n_seg = 1;
        c->seg_i0[0] = 0; c->seg_n[0] = ni; c->seg_dup[0] = 0;
    } else if (c->topo == FSI_TOPO_CGRID) {
        if (c->n_wake < 2 || ni - 2 * c->n_wake < 8)
            return fail(c, FSI_E_MESH, "C-grid needs n_wake >= 2 and at least 8 wall nodes");
        c->cut_a = -1; c->cut_b = c->n_wake; c->mirror = ni - 1;
        c->n_seg = 1;
        c->seg_i0[0] = c->n_wake; c->seg_n[0] = ni - 2 * c->n_wake; c->seg_dup[0] = 1;
    } else if (c->topo == FSI_TOPO_TWIN) {
        const int nA = ni - 2 * c->n_wake - c->n_wall2;
        if (c->n_wake < 2 || c->n_wall2 < 8 || nA < 8)
            return fail(c, FSI_E_MESH, "twin O-grid needs n_wake >= 2 slit cells and at least 8 "
                                       "wall cells round each body");
        c->cut_a = nA; c->cut_b = nA + c->n_wake; c->mirror = nA;
        c->n_seg = 2;
        c->seg_i0[0] = 0; c->seg_n[0] = nA + 1; c->seg_dup[0] = 1;
        c->seg_i0[1] = nA + c->n_wake; c->seg_n[1] = c->n_wall2 + 1; c->seg_dup[1] = 1;
    }
    return FSI_OK;
}

// unstructured 9-node mesh: connectivity, periodic offsets, node patches and
// element geometry; every element positively oriented at all nine nodes
// Blocks of U_BLOCK consecutive nodes for the LDS-staged interpolation: the
// elements holding a node of the block (every departure element of the
// block's nodes is one of them), the nodes of those elements (the block's
// halo), each element's nodes as halo positions and each node's own position.
// The block path is left off (empty tables) if the largest block's halo, element
// list and rest populations do not fit 64 KiB of LDS, or if FSILBM_UNSTRUCTURED_GATHER is
// set to "device" (k_u_collide and k_u_stream then go through device memory;
// both paths agree to FP32 rounding).
// planes of the departure tables: the eight moving directions, and with a
// moving body the rest direction (its point X + dt g^{-1} V_G moves with the mesh)
int q9_dep_planes(const fsi_ctx *c) {
    return !c->bodies.empty() && c->bodies[0].dof != FSI_DOF_FIXED ? 9 : 8;
}

void build_q9_blocks(fsi_ctx *c) {
    c->bh_off.clear(); c->bh_nodes.clear(); c->be_off.clear(); c->be_elem.clear();
    c->be_nodes.clear(); c->uself.clear();
    c->u_hmax = c->u_lemax = 0;
    const char *env = getenv("FSILBM_UNSTRUCTURED_GATHER");
    if (env && std::string(env) == "device") return;
    const int N = c->ni, nb = (N + fsi::U_BLOCK - 1) / fsi::U_BLOCK;
    std::vector<int> bh_off(nb + 1, 0), be_off(nb + 1, 0), bh_nodes, be_elem;
    std::vector<uint16_t> be_nodes, uself(N, 0);
    std::vector<int> els, nodes;
    int hmax = 0, lemax = 0;
    for (int b = 0; b < nb; ++b) {
        const int n0 = b * fsi::U_BLOCK, n1 = std::min(N, n0 + fsi::U_BLOCK);
        els.clear();
        for (int v = n0; v < n1; ++v)
            for (int q = c->patch_off[v]; q < c->patch_off[v + 1]; ++q) els.push_back(c->patch_ent[q] >> 4);
        std::sort(els.begin(), els.end());
        els.erase(std::unique(els.begin(), els.end()), els.end());
        nodes.clear();
        for (int e : els)
            for (int a = 0; a < 9; ++a) nodes.push_back(c->elems[9 * (size_t)e + a]);
        std::sort(nodes.begin(), nodes.end());
        nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
        if (nodes.size() > 65535) return;
        auto pos = [&](int v) {
            return (uint16_t)(std::lower_bound(nodes.begin(), nodes.end(), v) - nodes.begin());
        };
        for (int e : els) {
            be_elem.push_back(e);
            for (int a = 0; a < 16; ++a) be_nodes.push_back(a < 9 ? pos(c->elems[9 * (size_t)e + a]) : 0);
        }
        for (int v = n0; v < n1; ++v) uself[v] = pos(v);
        bh_nodes.insert(bh_nodes.end(), nodes.begin(), nodes.end());
        bh_off[b + 1] = (int)bh_nodes.size();
        be_off[b + 1] = (int)be_elem.size();
        hmax = std::max(hmax, (int)nodes.size());
        lemax = std::max(lemax, (int)els.size());
    }
    // the widest element stride that keeps four blocks per CU, else the
    // narrowest (a moving body stages the rest pair as a ninth plane)
    const int planes = q9_dep_planes(c);
    int eu16 = 10;
    for (int w : {16, 12, 10})
        if (fsi::u_block_lds_bytes(hmax, lemax, w, planes) <= fsi::U_LDS_PER_BLOCK) { eu16 = w; break; }
    if (fsi::u_block_lds_bytes(hmax, lemax, eu16, planes) > 65536) return;
    if (eu16 != 16) {
        std::vector<uint16_t> packed(be_nodes.size() / 16 * eu16, 0);
        for (size_t e = 0; e < be_nodes.size() / 16; ++e)
            for (int a = 0; a < 9; ++a) packed[e * eu16 + a] = be_nodes[e * 16 + a];
        be_nodes.swap(packed);
    }
    c->u_eu16 = eu16;
    c->bh_off.swap(bh_off); c->bh_nodes.swap(bh_nodes); c->be_off.swap(be_off);
    c->be_elem.swap(be_elem); c->be_nodes.swap(be_nodes); c->uself.swap(uself);
    c->u_hmax = hmax;
    c->u_lemax = lemax;
}

// Local coordinates (xi, eta) of the point at offset (px, py) from local node
// a of element e under the element's corner (first-order) map, by Newton in
// FP64 from the node's own position; false if the point is not in the element.
bool q9_locate_fp64(const fsi_ctx *c, int e, int a, double px, double py, double &xi, double &eta) {
    const int lp[9] = {-1, 1, 1, -1, 0, 1, 0, -1, 0}, lq[9] = {-1, -1, 1, 1, -1, 0, 1, 0, 0};
    const double *xy = c->ecoord.data() + 18 * (size_t)e;
    double cx[4], cy[4];
    for (int k = 0; k < 4; ++k) {
        cx[k] = xy[2 * k] - xy[2 * a];
        cy[k] = xy[2 * k + 1] - xy[2 * a + 1];
    }
    double u = lp[a], v = lq[a];
    for (int it = 0; it < 40; ++it) {
        const double n0 = (1 - u) * (1 - v), n1 = (1 + u) * (1 - v), n2 = (1 + u) * (1 + v), n3 = (1 - u) * (1 + v);
        const double rx = 0.25 * (n0 * cx[0] + n1 * cx[1] + n2 * cx[2] + n3 * cx[3]) - px;
        const double ry = 0.25 * (n0 * cy[0] + n1 * cy[1] + n2 * cy[2] + n3 * cy[3]) - py;
        const double ja = 0.25 * (-(1 - v) * cx[0] + (1 - v) * cx[1] + (1 + v) * cx[2] - (1 + v) * cx[3]);
        const double jb = 0.25 * (-(1 - u) * cx[0] - (1 + u) * cx[1] + (1 + u) * cx[2] + (1 - u) * cx[3]);
        const double jc = 0.25 * (-(1 - v) * cy[0] + (1 - v) * cy[1] + (1 + v) * cy[2] - (1 + v) * cy[3]);
        const double jd = 0.25 * (-(1 - u) * cy[0] - (1 + u) * cy[1] + (1 + u) * cy[2] + (1 - u) * cy[3]);
        const double det = ja * jd - jb * jc;
        const double du = (jd * rx - jb * ry) / det, dv = (-jc * rx + ja * ry) / det;
        u -= du;
        v -= dv;
        if (fabs(du) + fabs(dv) < 1e-14) break;
    }
    xi = u;
    eta = v;
    return fabs(u) <= 1.0 + 1e-12 && fabs(v) <= 1.0 + 1e-12;
}

// The body on a Q9 mesh: one fixed body with the mesh's wall polygon; the
// lumped normals (n ds)_k = rot90(x_{k+1} - x_{k-1}) / 2, the moment arms and
// the points B = x + dt n located in the wall node's elements (FP64).
fsi_status q9_wall_geometry(fsi_ctx *c) {
    const int nw = (int)c->qw_nodes.size();
    if ((int)c->bodies.size() != (nw > 0 ? 1 : 0))
        return fail(c, FSI_E_ARG, nw > 0 ? "a Q9 mesh with a wall polygon carries one body"
                                         : "a Q9 mesh without a wall polygon carries no body");
    c->qw_geo.clear();
    c->qw_eB.clear();
    c->qw_xyB.clear();
    c->qw_coff.assign(1, 0);
    c->qw_corner.clear();
    c->n_seg = 0;
    if (nw == 0) return FSI_OK;
    const fsi_body_desc &b = c->bodies[0];
    if (b.link >= 0) return fail(c, FSI_E_ARG, "a body on a Q9 mesh has no link");
    c->q9_moving = b.dof != FSI_DOF_FIXED;
    c->wall_dist.clear();
    if (c->q9_moving) {
        if (!(b.r_blend > b.r_rigid) || !(b.r_rigid >= 0))
            return fail(c, FSI_E_ARG, "a moving body on a Q9 mesh needs 0 <= r_rigid < r_blend");
        if (b.blend_mode != 0 && b.blend_mode != 1) return fail(c, FSI_E_ARG, "unknown blend_mode");
        const size_t N = (size_t)c->ni;
        if (b.blend_mode == 1) {
            // distance of every node to the closed wall polygon (undeformed frame)
            if ((double)N * (double)nw > 4e9)
                return fail(c, FSI_E_ARG, "distance blending: mesh too large for the direct "
                                          "distance computation (nodes x wall edges > 4e9)");
            c->wall_dist.assign(N, 0.0);
            for (size_t q = 0; q < N; ++q) {
                const double px = c->X[2 * q], py = c->X[2 * q + 1];
                double best = INFINITY;
                for (int e = 0; e < nw; ++e) {
                    const double *a = &c->X[2 * (size_t)c->qw_nodes[e]];
                    const double *bq = &c->X[2 * (size_t)c->qw_nodes[(e + 1) % nw]];
                    const double ex = bq[0] - a[0], ey = bq[1] - a[1];
                    const double ee = ex * ex + ey * ey;
                    double t = ee > 0 ? ((px - a[0]) * ex + (py - a[1]) * ey) / ee : 0.0;
                    t = t < 0 ? 0 : (t > 1 ? 1 : t);
                    const double dx = px - (a[0] + t * ex), dy = py - (a[1] + t * ey);
                    best = std::min(best, dx * dx + dy * dy);
                }
                c->wall_dist[q] = sqrt(best);
            }
        }
        // the blending coordinate of node v: the distance to the centre or
        // to the wall
        auto dist = [&](size_t v) {
            return b.blend_mode == 1 ? c->wall_dist[v]
                                     : hypot(c->X[2 * v] - b.center[0], c->X[2 * v + 1] - b.center[1]);
        };
        // the wall nodes' elements move rigidly with the body (B is placed
        // in the undeformed frame)
        for (int k = 0; k < nw; ++k) {
            const int v = c->qw_nodes[k];
            for (int q = c->patch_off[v]; q < c->patch_off[v + 1]; ++q) {
                const int e = c->patch_ent[q] >> 4;
                for (int a = 0; a < 9; ++a) {
                    const size_t u = (size_t)c->elems[9 * (size_t)e + a];
                    const double dw = b.blend_mode == 1 ? c->wall_dist[u] : 0.0;
                    if (blend_r(b, c->X[2 * u], c->X[2 * u + 1], dw) != 0.0)
                        return fail(c, FSI_E_ARG, "the elements at the wall must lie in the moving body's rigid zone "
                                                  "(r_rigid too small)");
                }
            }
        }
        // nodes the blending moves (Q9_MOVES: nearer than r_blend, with a
        // margin far above rounding) and nodes whose patch holds one
        // (Q9_PATCH_MOVES); the departure points of the others keep their
        // values of the undeformed mesh
        const double reach = b.r_blend * (1.0 + 1e-9);
        for (size_t v = 0; v < N; ++v)
            if (dist(v) < reach) c->qflag[v] |= fsi::Q9_MOVES;
        for (size_t v = 0; v < N; ++v)
            for (int q = c->patch_off[v]; q < c->patch_off[v + 1]; ++q) {
                const int e = c->patch_ent[q] >> 4;
                for (int a = 0; a < 9; ++a)
                    if (c->qflag[c->elems[9 * (size_t)e + a]] & fsi::Q9_MOVES) c->qflag[v] |= fsi::Q9_PATCH_MOVES;
            }
        // The displacement at level n+1 is (1 - r)(A X + b) with A = R(a) - I
        // and b = (0, h) - A X_EA of that level's body state, so its nodal
        // finite-element derivative (the mean over the node's elements of the
        // element derivative at the node) is, by linearity and the exactness
        // of that derivative for linear fields, A - A L[r X] - b (x) L[r] with
        // L[F] the nodal derivative of the static field F.  L[r], L[r X] and
        // L[r Y] are formed here once, in FP64 on the undeformed mesh.
        {
            const int lp[9] = {-1, 1, 1, -1, 0, 1, 0, -1, 0}, lq[9] = {-1, -1, 1, 1, -1, 0, 1, 0, 0};
            auto dl = [](int p, int x) { return p < 0 ? x - 0.5 : (p == 0 ? -2.0 * x : x + 0.5); };
            std::vector<double> rn(N), acc(6 * N, 0.0);
            for (size_t v = 0; v < N; ++v)
                rn[v] = blend_r(b, c->X[2 * v], c->X[2 * v + 1], b.blend_mode == 1 ? c->wall_dist[v] : 0.0);
            for (int e = 0; e < c->n_elems; ++e) {
                const double *xe = &c->ecoord[18 * (size_t)e];
                double F[3][9];
                for (int a = 0; a < 9; ++a) {
                    const size_t v = (size_t)c->elems[9 * (size_t)e + a];
                    F[0][a] = rn[v];
                    F[1][a] = rn[v] * c->X[2 * v];
                    F[2][a] = rn[v] * c->X[2 * v + 1];
                }
                for (int a = 0; a < 9; ++a) {
                    double xxi = 0, yxi = 0, xeta = 0, yeta = 0, fxi[3] = {}, feta[3] = {};
                    for (int m = -1; m <= 1; ++m) {
                        int si = -1, sj = -1;
                        for (int q = 0; q < 9; ++q) {
                            if (lp[q] == m && lq[q] == lq[a]) si = q;
                            if (lp[q] == lp[a] && lq[q] == m) sj = q;
                        }
                        const double wi = dl(m, lp[a]), wj = dl(m, lq[a]);
                        xxi += wi * (xe[2 * si] - xe[2 * a]);
                        yxi += wi * (xe[2 * si + 1] - xe[2 * a + 1]);
                        xeta += wj * (xe[2 * sj] - xe[2 * a]);
                        yeta += wj * (xe[2 * sj + 1] - xe[2 * a + 1]);
                        for (int f = 0; f < 3; ++f) {
                            fxi[f] += wi * (F[f][si] - F[f][a]);
                            feta[f] += wj * (F[f][sj] - F[f][a]);
                        }
                    }
                    const double idet = 1.0 / (xxi * yeta - yxi * xeta);
                    const size_t v = (size_t)c->elems[9 * (size_t)e + a];
                    for (int f = 0; f < 3; ++f) {
                        acc[6 * v + 2 * f] += idet * (yeta * fxi[f] - yxi * feta[f]);
                        acc[6 * v + 2 * f + 1] += idet * (-xeta * fxi[f] + xxi * feta[f]);
                    }
                }
            }
            // elements with a moving node, and elements wholly in the rigid
            // zone (a translation moves their nodes alike)
            c->q9_eflag.assign((size_t)c->n_elems, 0);
            for (int e = 0; e < c->n_elems; ++e) {
                bool moves = false, rigid = true;
                for (int a = 0; a < 9; ++a) {
                    const size_t v = (size_t)c->elems[9 * (size_t)e + a];
                    moves |= (c->qflag[v] & fsi::Q9_MOVES) != 0;
                    rigid &= rn[v] == 0.0;
                }
                c->q9_eflag[e] = (moves ? fsi::Q9E_MOVES : 0) | (rigid ? fsi::Q9E_RIGID : 0);
            }
            c->q9_dgr.assign(3 * N, make_float2(0.0f, 0.0f));
            for (size_t v = 0; v < N; ++v) {
                const double inv = 1.0 / (double)(c->patch_off[v + 1] - c->patch_off[v]);
                for (int f = 0; f < 3; ++f)
                    c->q9_dgr[3 * v + f] = make_float2((float)(acc[6 * v + 2 * f] * inv),
                                                       (float)(acc[6 * v + 2 * f + 1] * inv));
            }
        }
    }
    const double dt = c->fluid.dt;
    for (int k = 0; k < nw; ++k) {
        const int v = c->qw_nodes[k], vm = c->qw_nodes[(k + nw - 1) % nw], vp = c->qw_nodes[(k + 1) % nw];
        const double x = c->X[2 * (size_t)v], y = c->X[2 * (size_t)v + 1];
        const double nx = -0.5 * (c->X[2 * (size_t)vp + 1] - c->X[2 * (size_t)vm + 1]);
        const double ny = 0.5 * (c->X[2 * (size_t)vp] - c->X[2 * (size_t)vm]);
        c->qw_geo.push_back(make_double4(nx, ny, x - b.ea[0], y - b.ea[1]));
        const double nn = sqrt(nx * nx + ny * ny);
        if (!(nn > 0)) return fail(c, FSI_E_MESH, "degenerate Q9 wall polygon at wall node " + std::to_string(k));
        int eB = -1;
        double xi = 0, eta = 0;
        for (int q = c->patch_off[v]; q < c->patch_off[v + 1] && eB < 0; ++q) {
            const int ent = c->patch_ent[q];
            if (q9_locate_fp64(c, ent >> 4, ent & 15, dt * nx / nn, dt * ny / nn, xi, eta)) eB = ent >> 4;
        }
        if (eB < 0)
            return fail(c, FSI_E_MESH, "point B of Q9 wall node " + std::to_string(k) +
                                       " lies outside its elements (is the wall clockwise?)");
        c->qw_eB.push_back(eB);
        c->qw_xyB.push_back(make_float2((float)xi, (float)eta));
        for (int q = c->patch_off[v]; q < c->patch_off[v + 1]; ++q) {
            const int e = c->patch_ent[q] >> 4, a = c->patch_ent[q] & 15;
            const double *xy = c->ecoord.data() + 18 * (size_t)e;
            for (int m = 0; m < 4; ++m)
                c->qw_corner.push_back(make_double2(xy[2 * m] - xy[2 * a], xy[2 * m + 1] - xy[2 * a + 1]));
        }
        c->qw_coff.push_back((int)(c->qw_corner.size() / 4));
    }
    c->n_seg = 1;
    c->seg_i0[0] = 0;
    c->seg_n[0] = nw;
    c->seg_dup[0] = 0;
    return FSI_OK;
}

fsi_status validate_q9(fsi_ctx *c, const fsi_mesh_desc *mesh) {
    const int N = c->ni, E = mesh->n_elems;
    if (E < 1 || !mesh->elems || !mesh->elem_shifts)
        return fail(c, FSI_E_MESH, "Q9 mesh needs n_elems >= 1, elems and elem_shifts");
    const double Lx = c->shift_i[0], Ly = c->shift_j[1];
    bool shifted = false;
    for (size_t q = 0; q < 18 * (size_t)E; ++q) shifted = shifted || mesh->elem_shifts[q] != 0;
    if (shifted && (!(Lx > 0) || !(Ly > 0)))
        return fail(c, FSI_E_MESH, "a Q9 mesh with element shifts needs periods shift_i[0], shift_j[1] > 0");
    c->n_elems = E;
    c->elems.assign(mesh->elems, mesh->elems + 9 * (size_t)E);
    std::vector<int> count(N, 0);
    for (int e = 0; e < E; ++e)
        for (int a = 0; a < 9; ++a) {
            const int v = c->elems[9 * (size_t)e + a];
            const int sx = mesh->elem_shifts[18 * (size_t)e + 2 * a], sy = mesh->elem_shifts[18 * (size_t)e + 2 * a + 1];
            if (v < 0 || v >= N || sx < -1 || sx > 1 || sy < -1 || sy > 1)
                return fail(c, FSI_E_MESH, "Q9 element " + std::to_string(e) + ": node index or shift out of range");
            ++count[v];
        }
    for (int v = 0; v < N; ++v)
        if (!count[v]) return fail(c, FSI_E_MESH, "Q9 node " + std::to_string(v) + " belongs to no element");
    // boundary nodes
    c->qflag.assign(N, 0);
    c->qw_idx.assign(N, -1);
    c->qw_nodes.clear();
    c->qf_nodes.clear();
    if (mesh->n_wall_nodes < 0 || mesh->n_far_nodes < 0 || (mesh->n_wall_nodes > 0 && !mesh->wall_nodes) ||
        (mesh->n_far_nodes > 0 && !mesh->far_nodes))
        return fail(c, FSI_E_MESH, "Q9 boundary node lists missing");
    if (mesh->n_wall_nodes > 0 && mesh->n_wall_nodes < 3)
        return fail(c, FSI_E_MESH, "a Q9 wall polygon needs at least 3 nodes");
    for (int q = 0; q < mesh->n_wall_nodes + mesh->n_far_nodes; ++q) {
        const bool wall = q < mesh->n_wall_nodes;
        const int v = wall ? mesh->wall_nodes[q] : mesh->far_nodes[q - mesh->n_wall_nodes];
        if (v < 0 || v >= N || c->qflag[v])
            return fail(c, FSI_E_MESH, "Q9 boundary node out of range or listed twice");
        c->qflag[v] = wall ? fsi::Q9_WALL : fsi::Q9_FAR;
        if (wall) {
            c->qw_idx[v] = q;
            c->qw_nodes.push_back(v);
        } else {
            c->qf_nodes.push_back(v);
        }
    }
    // patches in element order
    c->patch_off.assign(N + 1, 0);
    for (int v = 0; v < N; ++v) c->patch_off[v + 1] = c->patch_off[v] + count[v];
    c->patch_ent.assign(9 * (size_t)E, 0);
    std::vector<int> fill(c->patch_off.begin(), c->patch_off.end() - 1);
    for (int e = 0; e < E; ++e)
        for (int a = 0; a < 9; ++a) c->patch_ent[fill[c->elems[9 * (size_t)e + a]]++] = e * 16 + a;
    // each node's first eight patch entries at a fixed stride, so that a
    // nodal mean reaches its elements in one memory round trip
    c->patch8.assign(8 * (size_t)N, -1);
    for (int v = 0; v < N; ++v)
        for (int j = 0; j < 8 && c->patch_off[v] + j < c->patch_off[v + 1]; ++j)
            c->patch8[8 * (size_t)v + j] = c->patch_ent[c->patch_off[v] + j];
    // geometry: FP64 unwrapped coordinates, offsets from the centre node in FP32
    const int lp[9] = {-1, 1, 1, -1, 0, 1, 0, -1, 0}, lq[9] = {-1, -1, 1, 1, -1, 0, 1, 0, 0};
    auto dl = [](int p, int x) { return p < 0 ? x - 0.5 : (p == 0 ? -2.0 * x : x + 0.5); };
    c->erel.assign(9 * (size_t)E, make_float2(0, 0));
    c->ecoord.assign(18 * (size_t)E, 0.0);
    for (int e = 0; e < E; ++e) {
        double x[9], y[9];
        for (int a = 0; a < 9; ++a) {
            const int v = c->elems[9 * (size_t)e + a];
            x[a] = c->X[2 * (size_t)v] + mesh->elem_shifts[18 * (size_t)e + 2 * a] * Lx;
            y[a] = c->X[2 * (size_t)v + 1] + mesh->elem_shifts[18 * (size_t)e + 2 * a + 1] * Ly;
            c->ecoord[18 * (size_t)e + 2 * a] = x[a];
            c->ecoord[18 * (size_t)e + 2 * a + 1] = y[a];
        }
        for (int a = 0; a < 9; ++a) c->erel[9 * (size_t)e + a] = make_float2((float)(x[a] - x[8]), (float)(y[a] - y[8]));
        // edge and centre nodes on the corners' bilinear map
        const int ca[4] = {0, 1, 2, 3}, cb[4] = {1, 2, 3, 0};
        const double h = fabs(x[1] - x[0]) + fabs(y[1] - y[0]) + fabs(x[3] - x[0]) + fabs(y[3] - y[0]);
        for (int k = 0; k < 4; ++k) {
            const double mx = 0.5 * (x[ca[k]] + x[cb[k]]), my = 0.5 * (y[ca[k]] + y[cb[k]]);
            if (fabs(x[4 + k] - mx) + fabs(y[4 + k] - my) > 1e-9 * h)
                return fail(c, FSI_E_MESH, "Q9 element " + std::to_string(e) + ": edge node off its edge's midpoint");
        }
        if (fabs(x[8] - 0.25 * (x[0] + x[1] + x[2] + x[3])) + fabs(y[8] - 0.25 * (y[0] + y[1] + y[2] + y[3])) > 1e-9 * h)
            return fail(c, FSI_E_MESH, "Q9 element " + std::to_string(e) + ": centre node off the corners' centre");
        // positive Jacobian at the nine nodes
        for (int a = 0; a < 9; ++a) {
            double xxi = 0, yxi = 0, xeta = 0, yeta = 0;
            for (int m = -1; m <= 1; ++m) {
                int si = -1, sj = -1;
                for (int b = 0; b < 9; ++b) {
                    if (lp[b] == m && lq[b] == lq[a]) si = b;
                    if (lp[b] == lp[a] && lq[b] == m) sj = b;
                }
                xxi += dl(m, lp[a]) * x[si];
                yxi += dl(m, lp[a]) * y[si];
                xeta += dl(m, lq[a]) * x[sj];
                yeta += dl(m, lq[a]) * y[sj];
            }
            if (!(xxi * yeta - yxi * xeta > 0))
                return fail(c, FSI_E_MESH, "Q9 element " + std::to_string(e) + ": det J <= 0 at a node");
        }
    }
    build_q9_blocks(c);
    return FSI_OK;
}

fsi_status validate_and_precompute(fsi_ctx *c) {
    const int ni = c->ni, nj = c->nj;
    if (c->topo == FSI_TOPO_Q9) return FSI_OK;    // validated by validate_q9
    fsi_status tst = topology(c);
    if (tst != FSI_OK) return tst;
    if (c->cut) {
        // row 0: every cut point and every duplicated wall point appears twice
        for (int i = std::max(c->cut_a, 0); i <= c->cut_b; ++i) {
            const int m = mirror_of(c, i);
            const double *a = &c->X[2 * (size_t)i], *b = &c->X[2 * (size_t)m];
            if (a[0] != b[0] || a[1] != b[1])
                return fail(c, FSI_E_MESH, "cut nodes (i, 0) and (mirror(i), 0) must coincide "
                                           "(first mismatch at i = " + std::to_string(i) + ")");
        }
    }
    // det(dX/dxi) > 0 everywhere (FE metric of the topology)
    for (int j = 0; j < nj; ++j) {
        for (int i = 0; i < ni; ++i) {
            double xi, yi, xe, ye;
            dX_di(c, i, j, xi, yi);
            dX_dj(c, i, j, xe, ye);
            const double det = xi * ye - yi * xe;
            if (!(det > 0))
                return fail(c, FSI_E_MESH, "det(dX/dxi) <= 0 at node (" + std::to_string(i) + ", " +
                                               std::to_string(j) + "): mesh must be right-handed");
        }
    }
    const int nb = (int)c->bodies.size();
    const size_t N = (size_t)ni * nj;
    bool any_dist = false;
    for (int k = 0; k < nb; ++k) {
        const fsi_body_desc &b = c->bodies[k];
        const std::string who = "body " + std::to_string(k) + ": ";
        if (b.link < -1 || b.link >= k || (b.link >= 0 && c->bodies[b.link].link != -1))
            return fail(c, FSI_E_ARG, who + "link must be -1 or an earlier body that is not linked");
        if (!(b.r_blend > b.r_rigid) || !(b.r_rigid >= 0))
            return fail(c, FSI_E_ARG, who + "needs 0 <= r_rigid < r_blend");
        if (b.blend_mode != 0 && b.blend_mode != 1) return fail(c, FSI_E_ARG, who + "unknown blend_mode");
        if (b.blend_mode == 1 && !c->has_wall)
            return fail(c, FSI_E_ARG, who + "distance blending needs a mesh with a wall");
        any_dist |= b.blend_mode == 1;
        if (b.link >= 0) continue;           // no equation of its own
        if (b.dof == FSI_DOF_HEAVE && !(b.m > 0)) return fail(c, FSI_E_ARG, who + "heave body needs m > 0");
        if (b.dof == FSI_DOF_PITCH_PLUNGE && !(b.m * b.I_a - b.S_a * b.S_a > 0))
            return fail(c, FSI_E_ARG, who + "pitch-plunge body needs a positive-definite mass matrix");
        if (!(b.release_time >= 0)) return fail(c, FSI_E_ARG, who + "release_time must be >= 0");
    }
    c->wall_dist.clear();
    if (any_dist) {
        // distance of every node to each distance-blended body's closed wall
        // polygon (undeformed frame); the polygons of the other bodies stay 0
        size_t E = 0;
        for (int k = 0; k < nb; ++k)
            if (c->bodies[k].blend_mode == 1) E += (size_t)(c->seg_n[k] - c->seg_dup[k]);
        if ((double)N * (double)E > 4e9)
            return fail(c, FSI_E_ARG, "distance blending: mesh too large for the direct "
                                      "distance computation (nodes x wall edges > 4e9)");
        c->wall_dist.assign((size_t)nb * N, 0.0);
        for (int k = 0; k < nb; ++k) {
            if (c->bodies[k].blend_mode != 1) continue;
            std::vector<int> poly;
            for (int i = 0; i < c->seg_n[k] - c->seg_dup[k]; ++i) poly.push_back(c->seg_i0[k] + i);
            const size_t Ek = poly.size();
            for (size_t q = 0; q < N; ++q) {
                const double px = c->X[2 * q], py = c->X[2 * q + 1];
                double best = INFINITY;
                for (size_t e = 0; e < Ek; ++e) {
                    const double *a = &c->X[2 * (size_t)poly[e]];
                    const double *bq = &c->X[2 * (size_t)poly[(e + 1) % Ek]];
                    const double ex = bq[0] - a[0], ey = bq[1] - a[1];
                    const double ee = ex * ex + ey * ey;
                    double t = ee > 0 ? ((px - a[0]) * ex + (py - a[1]) * ey) / ee : 0.0;
                    t = t < 0 ? 0 : (t > 1 ? 1 : t);
                    const double dx = px - (a[0] + t * ex), dy = py - (a[1] + t * ey);
                    best = std::min(best, dx * dx + dy * dy);
                }
                c->wall_dist[(size_t)k * N + q] = sqrt(best);
            }
        }
    }
    // regions of influence: at most one body moves a node
    if (nb > 1) {
        for (size_t q = 0; q < N; ++q) {
            int inside = 0;
            for (int k = 0; k < nb; ++k) {
                const double dw = c->wall_dist.empty() ? 0.0 : c->wall_dist[(size_t)k * N + q];
                if (blend_r(c->bodies[k], c->X[2 * q], c->X[2 * q + 1], dw) < 1.0) ++inside;
            }
            if (inside > 1)
                return fail(c, FSI_E_ARG, "regions of influence overlap at node (" +
                                              std::to_string(q % ni) + ", " + std::to_string(q / ni) + ")");
        }
    }
    if (c->topo == FSI_TOPO_PERIODIC2) {
        // a blended region must not reach the periodic seams
        for (int k = 0; k < nb; ++k)
            for (int j = 0; j < nj; ++j)
                for (int i = 0; i < ni; ++i) {
                    if (i > 3 && i < ni - 4 && j > 3 && j < nj - 4) continue;
                    const double *p = &c->X[2 * ((size_t)j * ni + i)];
                    if (blend_r(c->bodies[k], p[0], p[1]) < 1.0)
                        return fail(c, FSI_E_MESH, "blending region reaches a periodic seam");
                }
    }
    c->ff.clear();
    c->inflow.clear();
    c->wallB.assign(ni, make_float2(0, 0));
    if (c->has_wall) {
        const double dt = c->fluid.dt;
        for (int i = 0; i < ni; ++i) {
            if (!is_wall_col(c, i)) continue;
            double xp, yp, xm, ym, x0, y0;
            coord(c, i + 1, 0, xp, yp);
            coord(c, i - 1, 0, xm, ym);
            coord(c, i, 0, x0, y0);
            const double tx = xp - xm, ty = yp - ym, tn = hypot(tx, ty);
            const double bx = -ty / tn * dt, by = tx / tn * dt;   // B - X_A
            bool found = false;
            for (int di0 = -1; di0 <= 0 && !found; ++di0) {
                double cc[4][2];
                const int off[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
                for (int k = 0; k < 4; ++k) {
                    double x, y;
                    coord(c, i + di0 + off[k][0], off[k][1], x, y);
                    cc[k][0] = x - x0;
                    cc[k][1] = y - y0;
                }
                double s, t;
                if (bilinear_inverse(cc, bx, by, s, t) && s >= -1e-12 && s <= 1 + 1e-12 &&
                    t >= -1e-12 && t <= 1 + 1e-12) {
                    c->wallB[i] = make_float2((float)(di0 + s), (float)t);
                    found = true;
                }
            }
            if (!found)
                return fail(c, FSI_E_MESH, "wall point B (distance dt along the normal) leaves the "
                                           "first cell row at wall node " + std::to_string(i));
        }
        // far-field nodes: row nj - 1 (n_out = rot90(dX/di)), then the C-grid
        // exit columns (n_out = +-rot90(dX/dj)); inlet where u_inf . n_out < 0
        const double ux = c->fluid.u_inf[0], uy = c->fluid.u_inf[1];
        auto add = [&](int i, int j, double nx, double ny, int ir, int jr) {
            c->ff.push_back(make_int2(j * ni + i, jr * ni + ir));
            c->inflow.push_back((ux * nx + uy * ny) < 0.0 ? 1 : 0);
        };
        const bool cg = c->topo == FSI_TOPO_CGRID;     // exit columns
        for (int i = 0; i < ni; ++i) {
            double xd, yd;
            dX_di(c, i, nj - 1, xd, yd);
            add(i, nj - 1, -yd, xd, cg ? std::min(std::max(i, 1), ni - 2) : i, nj - 2);
        }
        if (cg) {
            for (int j = 0; j < nj - 1; ++j) {
                double xd, yd;
                dX_dj(c, 0, j, xd, yd);
                add(0, j, -yd, xd, 1, j);
                dX_dj(c, ni - 1, j, xd, yd);
                add(ni - 1, j, yd, -xd, ni - 2, j);
            }
        }
    }
    return FSI_OK;
}

// The fused kernel's tiles of an ni x nj instance on tile shape `shape`, as
// (instance, tile) work items in visiting order: `strips` column strips of
// equal width (the last one narrower), each strip row by row.
void append_tiles(std::vector<int2> &out, int inst, int ni, int nj, int shape, int strips) {
    const int tx = fsi::TILE_SHAPES[shape][0], ty = fsi::TILE_SHAPES[shape][1];
    const int tiles_i = (ni + tx - 1) / tx, tiles_j = (nj + ty - 1) / ty;
    const int w = (tiles_i + strips - 1) / strips;
    for (int s0 = 0; s0 < tiles_i; s0 += w)
        for (int tj = 0; tj < tiles_j; ++tj)
            for (int ti = s0; ti < std::min(s0 + w, tiles_i); ++ti) out.push_back(make_int2(inst, tj * tiles_i + ti));
}

void fill_params(fsi_ctx *c) {
    Inst &P = c->inst;
    const fsi_fluid_params &fl = c->fluid;
    P.ni = c->ni;
    P.nj = c->nj;
    P.periodic_j = c->topo == FSI_TOPO_PERIODIC2;
    P.cut = c->cut ? 1 : 0;
    P.exits = c->topo == FSI_TOPO_CGRID ? 1 : 0;
    P.cut_a = c->cut_a;
    P.cut_b = c->cut_b;
    P.mirror = c->mirror;
    P.exp_lo = std::max(c->cut_a, 0);
    P.cut_n = c->cut ? 2 * (c->cut_b - P.exp_lo + 1) : 0;
    P.n_seg = c->n_seg;
    for (int k = 0; k < fsi::MAX_BODIES; ++k) {
        P.seg_i0[k] = c->seg_i0[k];
        P.seg_n[k] = c->seg_n[k];
        P.seg_dup[k] = c->seg_dup[k];
    }
    P.n_ff = (int)c->ff.size();
    P.nbody = (int)c->bodies.size();
    P.n_sub = c->n_sub;
    P.relax = c->relax;
    P.storage = fl.storage;
    // 9-node meshes: non-temporal population stores where the step streams
    // more than the Infinity Cache holds (populations read and written, and
    // about 40 B per node of coordinates and departure data)
    P.stream_out = c->topo == FSI_TOPO_Q9 &&
                   (long long)c->ni * (2 * fsi::NPOP * (fl.storage == FSI_STORE_FP32 ? 4 : 2) + 40) > fsi::CACHE_BYTES;
    P.n_elems = c->n_elems;
    // 64 x 8 tiles and non-temporal population stores for meshes without a
    // cut and with at most one body whose step streams more than the
    // Infinity Cache holds; 32 x 16 otherwise
    {
        const long long pop_bytes = fl.storage == FSI_STORE_FP32 ? 4 : 2;
        const long long step_bytes = (long long)c->ni * c->nj * (2 * fsi::NPOP * pop_bytes + 16);
        c->stream_out = !c->cut && c->bodies.size() <= 1 && step_bytes > fsi::CACHE_BYTES;
        c->shape = c->stream_out ? fsi::WIDE_SHAPE : 0;
    }
    const int sx = fsi::TILE_SHAPES[c->shape][0], sy = fsi::TILE_SHAPES[c->shape][1];
    P.tiles_i = (c->ni + sx - 1) / sx;
    P.tiles_j = (c->nj + sy - 1) / sy;
    P.tile_base = 0;
    P.n_nodes = (long long)c->ni * c->nj;
    P.shift_ix = c->shift_i[0];
    P.shift_iy = c->shift_i[1];
    P.shift_jx = c->shift_j[0];
    P.shift_jy = c->shift_j[1];
    P.dt_d = fl.dt;
    P.gm1_d = fl.gamma - 1.0;
    P.gamma = (float)fl.gamma;
    const double Cv = 1.0 / (fl.gamma - 1.0);
    P.Cv = (float)Cv;
    P.Cp = (float)(Cv + 1.0);
    P.mu = (float)fl.mu;
    P.Pr = (float)fl.Pr;
    P.dt = (float)fl.dt;
    P.rho_inf = (float)fl.rho_inf;
    P.T_inf = (float)fl.T_inf;
    P.ux_inf = (float)fl.u_inf[0];
    P.uy_inf = (float)fl.u_inf[1];
    // FP16 shifted storage: reference = free-stream equilibrium populations
    {
        const double rho = fl.rho_inf, ux = fl.u_inf[0], uy = fl.u_inf[1], T = fl.T_inf;
        const double E = Cv * T + 0.5 * (ux * ux + uy * uy);
        const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        auto phi = [&](int cc, double u) { return cc == 0 ? 1 - (u * u + T) : 0.5 * (cc * u + u * u + T); };
        auto w1 = [&](int cc) { return cc == 0 ? 1 - T : 0.5 * T; };
        for (int k = 0; k < 9; ++k) {
            P.ref[k] = (float)(rho * phi(cx[k], ux) * phi(cy[k], uy));
            P.ref[9 + k] = (float)(2.0 * rho * E * w1(cx[k]) * w1(cy[k]));
        }
        P.scale[0] = 1.0f / 64.0f;
        P.scale[1] = 1.0f / 16.0f;
        P.inv_scale[0] = 64.0f;
        P.inv_scale[1] = 16.0f;
    }
    for (int k = 0; k < fsi::MAX_BODIES; ++k) {
        fsi::Body &B = P.body[k];
        B = fsi::Body{};
        B.master = k;
        B.dof = fsi::DOF_FIXED;
        if (k >= (int)c->bodies.size()) continue;
        const fsi_body_desc &b = c->bodies[k];
        // a linked body moves with its master's rigid map and state
        const int m = b.link >= 0 ? b.link : k;
        const fsi_body_desc &bm = c->bodies[m];
        B.present = 1;
        B.master = m;
        B.dof = bm.dof;
        B.m = bm.m; B.S_a = bm.S_a; B.I_a = bm.I_a; B.k_h = bm.k_h; B.k_a = bm.k_a;
        B.cx = b.center[0]; B.cy = b.center[1]; B.ex = bm.ea[0]; B.ey = bm.ea[1];
        B.r_rigid = b.r_rigid;
        B.inv_width = 1.0 / (b.r_blend - b.r_rigid);
        B.r_rigid2 = b.r_rigid > 0.0 ? b.r_rigid * b.r_rigid : -1.0;
        B.r_blend2 = b.r_blend * b.r_blend;
        B.heave_amp = bm.heave_amp; B.heave_omega = 2.0 * M_PI * bm.heave_freq;
        B.pitch_amp = bm.pitch_amp; B.pitch_omega = 2.0 * M_PI * bm.pitch_freq;
        B.release_time = bm.release_time;
        B.blend_mode = b.blend_mode;
    }
    // work lists
    c->wk1.clear();
    if (c->topo != FSI_TOPO_Q9) append_tiles(c->wk1, 0, c->ni, c->nj, c->shape, fsi::N_XCD);
    c->wk1s.clear();
    c->n_near = 0;
    if (c->topo == FSI_TOPO_OGRID) {
        const int ty = fsi::TILE_SHAPES[c->shape][1];
        auto near = [&](int2 w) {
            const int j0 = (w.y / P.tiles_i) * ty, j1 = std::min(j0 + ty, c->nj) - 1;
            return j0 <= 2 || j1 >= c->nj - 2;
        };
        for (int2 w : c->wk1)
            if (near(w)) c->wk1s.push_back(w);
        c->n_near = (int)c->wk1s.size();
        // the interior tiles in strip order: one strip per XCD as before
        std::vector<int2> far;
        append_tiles(far, 0, c->ni, c->nj, c->shape, fsi::N_XCD);
        for (int2 w : far)
            if (!near(w)) c->wk1s.push_back(w);
    }
    // only where the interior launch outlasts the boundary kernels by far: a
    // step that streams more than the Infinity Cache (a small instance's step
    // is launch-bound, and the second stream's fork and join would cost more
    // than the overlap saves)
    c->split = c->stream_out && c->n_near > 0 && c->n_near < (int)c->wk1s.size();
    c->wbnd.clear();
    c->wwall.clear();
    c->wk0.clear();
    if (c->has_wall) {
        int nw = 0;
        for (int k = 0; k < c->n_seg; ++k) nw += (c->seg_n[k] + 63) / 64;
        const int nf = (P.n_ff + 63) / 64;
        for (int b = 0; b < nw; ++b) {
            c->wbnd.push_back(make_int2(0, 2 * b));
            c->wwall.push_back(make_int2(0, b));
        }
        for (int b = 0; b < nf; ++b) c->wbnd.push_back(make_int2(0, 2 * b + 1));
    }
    if (c->cut) {
        // tiles of row block 0 that own a column whose row-1 state crosses
        // the cut (exported primary columns and their mirror images)
        for (int ti = 0; ti < P.tiles_i; ++ti) {
            const int a = ti * fsi::TILE_X, b = std::min(a + fsi::TILE_X, c->ni) - 1;
            bool own = false;
            for (int i = a; i <= b && !own; ++i) {
                const int m = mirror_of(c, i);
                own = (i >= P.exp_lo && i <= c->cut_b) || (m >= P.exp_lo && m <= c->cut_b);
            }
            if (own) c->wk0.push_back(make_int2(0, ti));
        }
    }
}

void layout(fsi_ctx *c) {
    const size_t N = (size_t)c->ni * c->nj;
    const size_t bpp = c->fluid.storage == FSI_STORE_FP16_SHIFTED ? 2 : 4;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + std::max<size_t>(bytes, 1)); return r; };
    c->off_pop[0] = take(fsi::NPOP * N * bpp);
    c->off_pop[1] = take(fsi::NPOP * N * bpp);
    c->off_X = take(N * 16);
    c->off_mask = take(c->ni * 4);                 // missing mask, then the ambiguity mask
    c->off_tgt = take(c->ni * 16);
    c->off_B = take(c->ni * 8);
    c->off_inflow = take(c->ff.size());
    c->off_ff = take(c->ff.size() * sizeof(int2));
    c->off_cut = take((size_t)18 * c->inst.cut_n * sizeof(float));
    c->off_force = take(c->ni * 32);
    c->off_slots = take(3 * fsi::MAX_BODIES * sizeof(fsi::BodySlot));
    c->off_hist = take((size_t)fsi::MAX_BODIES * fsi::HIST_CAP * 6 * 8);
    c->off_step = take(8);
    c->off_err = take(4);
    c->off_inst = take(sizeof(Inst));
    c->off_inst_na = take(sizeof(Inst));
    c->off_wk1 = take(c->wk1.size() * sizeof(int2));
    c->off_wk1s = take(c->wk1s.size() * sizeof(int2));
    c->off_wbnd = take(c->wbnd.size() * sizeof(int2));
    c->off_wwall = take(c->wwall.size() * sizeof(int2));
    c->off_wk0 = take(c->wk0.size() * sizeof(int2));
    c->off_dist = take(c->wall_dist.size() * sizeof(double));
    c->off_resid = take(fsi::MAX_BODIES * sizeof(double));
    if (c->topo == FSI_TOPO_Q9) {
        c->off_elems = take(c->elems.size() * 4);
        c->off_erel = take(c->erel.size() * sizeof(float2));
        c->off_poff = take(c->patch_off.size() * 4);
        c->off_pent = take(c->patch_ent.size() * 4);
        c->off_uq = take(N * sizeof(float2));
        c->off_us = take(N * sizeof(float));
        c->off_ud = take(N * sizeof(float2));
        c->off_ueg = take(9 * (size_t)c->n_elems * sizeof(float2));
        const size_t planes = (size_t)q9_dep_planes(c);
        c->off_upost = take(2 * planes * N * sizeof(float));
        c->off_dep_e = take(planes * N * 4);
        c->off_dep_xy = take(planes * N * sizeof(float2));
        c->off_qflag = take(N);
        c->off_qwidx = take(N * 4);
        c->off_qw = take(c->qw_nodes.size() * 4);
        c->off_qf = take(c->qf_nodes.size() * 4);
        c->off_qwgeo = take(c->qw_geo.size() * sizeof(double4));
        c->off_qweB = take(c->qw_eB.size() * 4);
        c->off_qwxyB = take(c->qw_xyB.size() * sizeof(float2));
        c->off_qwcoff = take(c->qw_coff.size() * 4);
        c->off_qwcorner = take(c->qw_corner.size() * sizeof(double2));
        c->off_qwprev = take(c->qw_nodes.size() * sizeof(float2));
        if (c->q9_moving) {
            c->off_qdisp = take(2 * N * sizeof(double2));
            c->off_dgr = take(c->q9_dgr.size() * sizeof(float2));
            c->off_eflag = take(c->q9_eflag.size());
        }
        c->off_patch8 = take(c->patch8.size() * 4);
        if (!c->bh_off.empty()) {
            c->off_bh_off = take(c->bh_off.size() * 4);
            c->off_bh_nodes = take(c->bh_nodes.size() * 4);
            c->off_be_off = take(c->be_off.size() * 4);
            c->off_be_elem = take(c->be_elem.size() * 4);
            c->off_be_nodes = take(c->be_nodes.size() * 2);
            c->off_uself = take(c->uself.size() * 2);
            c->off_dep_le = take(planes * N * 2);
        }
    }
    c->total = o;
}

fsi_status check_ready(fsi_ctx *c, bool need_init) {
    if (!c) return FSI_E_ARG;
    if (!c->ws) return fail(c, FSI_E_UNBOUND, "workspace not bound");
    if (need_init && !c->initialized) return fail(c, FSI_E_UNBOUND, "state not initialised");
    return FSI_OK;
}

const Inst *d_inst(fsi_ctx *c) { return reinterpret_cast<const Inst *>(c->ws + c->off_inst); }
const Inst *d_inst_na(fsi_ctx *c) { return reinterpret_cast<const Inst *>(c->ws + c->off_inst_na); }

// The instance copy of fsi_step_noalloc: the bound instance with its per-step
// scratch (wall masks, targets, tractions, cut staging) in the static scratch
// array of the current device.  Structured meshes whose scratch fits the
// array only (else na_bytes stays 0 and the entry point refuses).
fsi_status upload_inst_na(fsi_ctx *c) {
    c->na_ready = false;
    c->na_bytes = 0;
    if (c->topo == FSI_TOPO_Q9) return FSI_OK;
    size_t off[5];
    const size_t need = na_layout(c, off);
    if (need > kNoAllocScratchBytes) return FSI_OK;
    void *base = nullptr;
    HIP_TRY(c, noalloc_scratch(&base));
    char *sb = static_cast<char *>(base);
    Inst P = c->inst;
    P.wall_mask = reinterpret_cast<uint16_t *>(sb + off[0]);
    P.wall_amb = P.wall_mask + c->ni;
    P.wall_tgt = reinterpret_cast<float4 *>(sb + off[1]);
    P.wall_force = reinterpret_cast<double4 *>(sb + off[2]);
    P.cutbuf = reinterpret_cast<float *>(sb + off[3]);
    HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_inst_na, &P, sizeof(Inst), hipMemcpyHostToDevice, c->stream));
    c->na_bytes = need;
    c->na_ready = true;
    return FSI_OK;
}

// one pass of the fluid part of a step on the populations of level n: the cut
// pre-pass, collision-streaming, wall targets and far field, Grad populations
// and traction of the new level
fsi_status enqueue_fluid(fsi_ctx *c, const Inst *di, bool split) {
    const int st = c->fluid.storage;
    if (c->topo == FSI_TOPO_Q9) {
        // a moving body: the mesh of both levels and the departure points on
        // it (relocated by the node-block kernel itself where it runs)
        const bool fused = c->q9_moving && c->inst.u_nblk > 0;
        if (c->q9_moving)
            HIP_TRY(c, fsi::launch_unstructured_motion(d_inst(c), (long long)c->ni, (long long)c->n_elems,
                                                       fused ? 0 : 1, c->stream));
        HIP_TRY(c, fsi::launch_unstructured(d_inst(c), (long long)c->ni, (long long)c->n_elems, st,
                                            c->inst.uq, c->inst.ud, c->inst.ueg, c->inst.u_nblk,
                                            c->inst.u_hmax, c->inst.u_lemax, c->inst.u_eu16, c->inst.qdisp,
                                            fused ? 1 : 0, c->stream));
        if (!c->qw_nodes.empty() || !c->qf_nodes.empty())
            HIP_TRY(c, fsi::launch_unstructured_boundary(d_inst(c), (int)c->qw_nodes.size(),
                                                         (int)c->qf_nodes.size(), st, 1, c->stream));
        return FSI_OK;
    }
    if (!c->wk0.empty())
        HIP_TRY(c, fsi::launch_cut_export(di, reinterpret_cast<const int2 *>(c->ws + c->off_wk0),
                                          (int)c->wk0.size(), st, c->stream));
    if (split) {
        // interior tiles on the second stream, from the state the step starts
        // from; they read and write nothing the boundary kernels touch
        const int2 *wk1s = reinterpret_cast<const int2 *>(c->ws + c->off_wk1s);
        HIP_TRY(c, hipEventRecord(c->ev_fork, c->stream));
        HIP_TRY(c, hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
        HIP_TRY(c, fsi::launch_collide_stream(di, wk1s + c->n_near, (int)c->wk1s.size() - c->n_near, st,
                                              c->stream2, 0, c->cut, c->shape, c->stream_out));
        HIP_TRY(c, hipEventRecord(c->ev_join, c->stream2));
        HIP_TRY(c, fsi::launch_collide_stream(di, wk1s, c->n_near, st, c->stream, 0, c->cut, c->shape,
                                              c->stream_out));
    } else {
        HIP_TRY(c, fsi::launch_collide_stream(di, reinterpret_cast<const int2 *>(c->ws + c->off_wk1),
                                              (int)c->wk1.size(), st, c->stream, 0, c->cut, c->shape,
                                              c->stream_out));
    }
    if (c->has_wall) {
        HIP_TRY(c, fsi::launch_wall_targets(di, reinterpret_cast<const int2 *>(c->ws + c->off_wbnd),
                                            (int)c->wbnd.size(), st, c->stream));
        HIP_TRY(c, fsi::launch_wall_grad_force(di,
                                               reinterpret_cast<const int2 *>(c->ws + c->off_wwall),
                                               (int)c->wwall.size(), st, 1, c->stream));
    }
    // every tile has read the step counter before the body kernel advances it
    if (split) HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
    return FSI_OK;
}

// one coupled step: with strong coupling, n_sub - 1 sub-iterations (fluid pass,
// structure re-solved and relaxed) before the final pass, which the body
// kernel accepts and records
fsi_status enqueue_step(fsi_ctx *c, const Inst *di = nullptr, bool split = false) {
    if (!di) di = d_inst(c);
    // without a body there is nothing to iterate on: one pass
    const int passes = c->bodies.empty() ? 1 : c->n_sub;
    for (int k = 0; k < passes; ++k) {
        if (k > 0 && c->topo == FSI_TOPO_Q9) {
            // an unstructured pass overwrote the moments of level n (the next
            // step's, formed by its interpolation) and the wall nodes' (rho, T)
            // of level n: form them again from the populations of level n
            HIP_TRY(c, fsi::launch_unstructured_moments(d_inst(c), (long long)c->ni, c->fluid.storage, c->stream));
            if (!c->qw_nodes.empty())
                HIP_TRY(c, fsi::launch_unstructured_boundary(d_inst(c), (int)c->qw_nodes.size(), 0,
                                                             c->fluid.storage, 0, c->stream));
        }
        fsi_status st = enqueue_fluid(c, di, split);
        if (st != FSI_OK) return st;
        HIP_TRY(c, fsi::launch_body(di, 1, k + 1 < passes ? 2 : 1, c->stream));
    }
    return FSI_OK;
}

// force of the current level and the next body state (no boundary update)
fsi_status enqueue_load_update(fsi_ctx *c) {
    // unstructured meshes: the moments the next step's correction starts from
    // (each step's interpolation forms them for the populations it writes)
    if (c->topo == FSI_TOPO_Q9) {
        HIP_TRY(c, fsi::launch_unstructured_moments(d_inst(c), (long long)c->ni, c->fluid.storage, c->stream));
        if (c->q9_moving)
            HIP_TRY(c, fsi::launch_unstructured_motion(d_inst(c), (long long)c->ni, (long long)c->n_elems, 0,
                                                       c->stream));
        if (!c->qw_nodes.empty())
            HIP_TRY(c, fsi::launch_unstructured_boundary(d_inst(c), (int)c->qw_nodes.size(), 0,
                                                         c->fluid.storage, 0, c->stream));
    }
    if (c->has_wall)
        HIP_TRY(c, fsi::launch_wall_grad_force(d_inst(c),
                                               reinterpret_cast<const int2 *>(c->ws + c->off_wwall),
                                               (int)c->wwall.size(), c->fluid.storage, 0, c->stream));
    HIP_TRY(c, fsi::launch_body(d_inst(c), 1, 0, c->stream));
    return FSI_OK;
}

fsi_status sync_check(fsi_ctx *c) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    unsigned e = 0;
    HIP_TRY(c, hipMemcpy(&e, c->ws + c->off_err, 4, hipMemcpyDeviceToHost));
    if (e & fsi::ERR_STATE) return fail(c, FSI_E_STATE, "non-physical state (rho<=0, T<=0, T+u^2>=1 or NaN)");
    if (e & fsi::ERR_CFL) return fail(c, FSI_E_CFL, "departure point outside the cells around its node");
    if (e & fsi::ERR_MESH) return fail(c, FSI_E_MESH, "inverted cell after mesh blending");
    return FSI_OK;
}

void drop_graph(fsi_ctx *c) {
    for (int q = 0; q < 2; ++q) {
        // teardown: a failure here leaves nothing to undo
        if (c->graph_exec[q]) (void)hipGraphExecDestroy(c->graph_exec[q]);
        if (c->graph[q]) (void)hipGraphDestroy(c->graph[q]);
        c->graph_exec[q] = nullptr;
        c->graph[q] = nullptr;
    }
}

// Steps per replay of the long graph: a graph launch costs a few microseconds
// between steps, kernels inside one graph follow each other without a gap.
constexpr int kGraphSteps = 16;

// capture `count` steps into graph slot q
fsi_status capture_steps(fsi_ctx *c, int q, int count) {
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    fsi_status st = FSI_OK;
    for (int k = 0; k < count && st == FSI_OK; ++k) st = enqueue_step(c, nullptr, c->stream2 != nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (st != FSI_OK) {
        if (g) (void)hipGraphDestroy(g);   // the capture's own error is reported
        return st;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    c->graph[q] = g;
    HIP_TRY(c, hipGraphInstantiate(&c->graph_exec[q], g, nullptr, nullptr, 0));
    return FSI_OK;
}

}  // namespace

extern "C" {

int64_t fsi_history_capacity(void) { return fsi::HIST_CAP; }

fsi_status fsi_create(const fsi_fluid_params *fluid, const fsi_mesh_desc *mesh,
                      const fsi_body_desc *bodies, int nbodies, void *hip_stream, fsi_ctx **out) {
    if (!out) return FSI_E_ARG;
    *out = nullptr;
    if (!fluid || !mesh || !mesh->X) return FSI_E_ARG;
    fsi_ctx *c = new (std::nothrow) fsi_ctx();
    if (!c) return FSI_E_NOMEM;
    *out = c;
    c->fluid = *fluid;
    c->ni = mesh->ni;
    c->nj = mesh->nj;
    c->topo = mesh->topo;
    c->n_wake = mesh->n_wake;
    c->n_wall2 = mesh->n_wall2;
    c->has_wall = c->topo == FSI_TOPO_OGRID || c->topo == FSI_TOPO_CGRID || c->topo == FSI_TOPO_TWIN;
    c->stream = (hipStream_t)hip_stream;
    if (c->topo != FSI_TOPO_PERIODIC2 && c->topo != FSI_TOPO_OGRID && c->topo != FSI_TOPO_CGRID &&
        c->topo != FSI_TOPO_TWIN && c->topo != FSI_TOPO_Q9)
        return fail(c, FSI_E_ARG, "unsupported topology");
    if (c->topo == FSI_TOPO_Q9 ? (c->ni < 9 || c->nj != 1) : (c->ni < 8 || c->nj < 8))
        return fail(c, FSI_E_ARG, c->topo == FSI_TOPO_Q9 ? "a Q9 mesh has ni = nodes >= 9 and nj = 1"
                                                         : "mesh needs ni >= 8 and nj >= 8");
    if (c->topo == FSI_TOPO_Q9 && nbodies > 1) return fail(c, FSI_E_ARG, "a Q9 mesh carries at most one body");
    if (c->topo == FSI_TOPO_TWIN ? nbodies != fsi::MAX_BODIES : (nbodies < 0 || nbodies > 1))
        return fail(c, FSI_E_ARG, c->topo == FSI_TOPO_TWIN ? "a twin O-grid carries 2 bodies"
                                                           : "nbodies must be 0 or 1");
    if (nbodies > 0 && !bodies) return fail(c, FSI_E_ARG, "bodies missing");
    if (!(fluid->gamma > 1) || !(fluid->mu > 0) || !(fluid->dt > 0) || !(fluid->Pr > 0) ||
        !(fluid->rho_inf > 0) || !(fluid->T_inf > 0 && fluid->T_inf < 1))
        return fail(c, FSI_E_ARG, "fluid parameters out of range");
    if (fluid->storage != FSI_STORE_FP32 && fluid->storage != FSI_STORE_FP16_SHIFTED)
        return fail(c, FSI_E_ARG, "unknown storage mode");
    if ((long long)c->ni * c->nj * fsi::NPOP * 4 >= (1LL << 31))
        return fail(c, FSI_E_ARG, "mesh too large: the kernels address each population array "
                                  "with 32-bit offsets (18 * 4 * ni * nj < 2^31, ~29.8M nodes)");
    for (int k = 0; k < 2; ++k) {
        c->shift_i[k] = mesh->shift_i[k];
        c->shift_j[k] = mesh->shift_j[k];
    }
    if (c->topo != FSI_TOPO_PERIODIC2 && c->topo != FSI_TOPO_Q9)
        c->shift_i[0] = c->shift_i[1] = c->shift_j[0] = c->shift_j[1] = 0;
    c->X.assign(mesh->X, mesh->X + 2 * (size_t)c->ni * c->nj);
    for (double v : c->X)
        if (!isfinite(v)) return fail(c, FSI_E_MESH, "non-finite mesh coordinate");
    for (int k = 0; k < nbodies; ++k) {
        c->bodies.push_back(bodies[k]);
        if ((bodies[k].link < 0 && (bodies[k].dof < 0 || bodies[k].dof > 3)))
            return fail(c, FSI_E_ARG, "unknown body dof");
    }
    if (c->topo == FSI_TOPO_Q9) {
        fsi_status sq = validate_q9(c, mesh);
        if (sq != FSI_OK) return sq;
        sq = q9_wall_geometry(c);
        if (sq != FSI_OK) return sq;
    }
    fsi_status st = validate_and_precompute(c);
    if (st != FSI_OK) return st;
    fill_params(c);
    layout(c);
    return FSI_OK;
}

fsi_status fsi_workspace_bytes(const fsi_ctx *c, size_t *bytes) {
    if (!c || !bytes) return FSI_E_ARG;
    *bytes = c->total;
    return FSI_OK;
}

fsi_status fsi_bind_workspace(fsi_ctx *c, void *dev_ptr, size_t bytes) {
    if (!c || !dev_ptr) return FSI_E_ARG;
    if (((uintptr_t)dev_ptr & 255) != 0) return fail(c, FSI_E_ARG, "workspace must be 256-byte aligned");
    if (bytes < c->total) return fail(c, FSI_E_ARG, "workspace too small");
    drop_graph(c);
    c->ws = static_cast<char *>(dev_ptr);
    c->initialized = false;
    Inst &P = c->inst;
    P.pop[0] = c->ws + c->off_pop[0];
    P.pop[1] = c->ws + c->off_pop[1];
    P.X = reinterpret_cast<const double2 *>(c->ws + c->off_X);
    P.wall_mask = reinterpret_cast<uint16_t *>(c->ws + c->off_mask);
    P.wall_amb = P.wall_mask + c->ni;
    P.wall_tgt = reinterpret_cast<float4 *>(c->ws + c->off_tgt);
    P.wall_B = reinterpret_cast<const float2 *>(c->ws + c->off_B);
    P.inflow = reinterpret_cast<const uint8_t *>(c->ws + c->off_inflow);
    P.ff = reinterpret_cast<const int2 *>(c->ws + c->off_ff);
    P.cutbuf = reinterpret_cast<float *>(c->ws + c->off_cut);
    P.wall_dist = c->wall_dist.empty() ? nullptr : reinterpret_cast<const double *>(c->ws + c->off_dist);
    if (!c->wall_dist.empty())
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_dist, c->wall_dist.data(), c->wall_dist.size() * 8,
                                  hipMemcpyHostToDevice, c->stream));
    P.wall_force = reinterpret_cast<double4 *>(c->ws + c->off_force);
    P.slots = reinterpret_cast<fsi::BodySlot *>(c->ws + c->off_slots);
    P.history = reinterpret_cast<double *>(c->ws + c->off_hist);
    P.resid = reinterpret_cast<double *>(c->ws + c->off_resid);
    if (c->topo == FSI_TOPO_Q9) {
        P.elems = reinterpret_cast<const int *>(c->ws + c->off_elems);
        P.erel = reinterpret_cast<const float2 *>(c->ws + c->off_erel);
        P.patch_off = reinterpret_cast<const int *>(c->ws + c->off_poff);
        P.patch_ent = reinterpret_cast<const int *>(c->ws + c->off_pent);
        P.uq = reinterpret_cast<float2 *>(c->ws + c->off_uq);
        P.us = reinterpret_cast<float *>(c->ws + c->off_us);
        P.ud = reinterpret_cast<float2 *>(c->ws + c->off_ud);
        P.ueg = reinterpret_cast<float2 *>(c->ws + c->off_ueg);
        P.upost = c->ws + c->off_upost;
        P.dep_e = reinterpret_cast<int *>(c->ws + c->off_dep_e);
        P.dep_xy = reinterpret_cast<float2 *>(c->ws + c->off_dep_xy);
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_elems, c->elems.data(), c->elems.size() * 4,
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_erel, c->erel.data(), c->erel.size() * sizeof(float2),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_poff, c->patch_off.data(), c->patch_off.size() * 4,
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_pent, c->patch_ent.data(), c->patch_ent.size() * 4,
                                  hipMemcpyHostToDevice, c->stream));
        P.n_qw = (int)c->qw_nodes.size();
        {
            const fsi_body_desc *bd = c->bodies.empty() ? nullptr : &c->bodies[0];
            P.q9_rotates = c->q9_moving && bd &&
                           (bd->dof == FSI_DOF_PITCH_PLUNGE || bd->a0 != 0.0 || bd->ad0 != 0.0 ||
                            bd->pitch_amp != 0.0);
        }
        P.n_qf = (int)c->qf_nodes.size();
        P.qflag = reinterpret_cast<const uint8_t *>(c->ws + c->off_qflag);
        P.qw_idx = reinterpret_cast<const int *>(c->ws + c->off_qwidx);
        P.qw_nodes = reinterpret_cast<const int *>(c->ws + c->off_qw);
        P.qf_nodes = reinterpret_cast<const int *>(c->ws + c->off_qf);
        P.qw_geo = reinterpret_cast<const double4 *>(c->ws + c->off_qwgeo);
        P.qw_eB = reinterpret_cast<const int *>(c->ws + c->off_qweB);
        P.qw_xyB = reinterpret_cast<const float2 *>(c->ws + c->off_qwxyB);
        P.qw_coff = reinterpret_cast<const int *>(c->ws + c->off_qwcoff);
        P.qw_corner = reinterpret_cast<const double2 *>(c->ws + c->off_qwcorner);
        P.qw_prev = reinterpret_cast<float2 *>(c->ws + c->off_qwprev);
        P.qdisp = c->q9_moving ? reinterpret_cast<double2 *>(c->ws + c->off_qdisp) : nullptr;
        P.dgr = c->q9_moving ? reinterpret_cast<const float2 *>(c->ws + c->off_dgr) : nullptr;
        P.eflag = c->q9_moving ? reinterpret_cast<const uint8_t *>(c->ws + c->off_eflag) : nullptr;
        P.patch8 = reinterpret_cast<const int *>(c->ws + c->off_patch8);
        {
            const std::pair<size_t, std::pair<const void *, size_t>> up[] = {
                {c->off_qflag, {c->qflag.data(), c->qflag.size()}},
                {c->off_qwidx, {c->qw_idx.data(), c->qw_idx.size() * 4}},
                {c->off_qw, {c->qw_nodes.data(), c->qw_nodes.size() * 4}},
                {c->off_qf, {c->qf_nodes.data(), c->qf_nodes.size() * 4}},
                {c->off_qwgeo, {c->qw_geo.data(), c->qw_geo.size() * sizeof(double4)}},
                {c->off_qweB, {c->qw_eB.data(), c->qw_eB.size() * 4}},
                {c->off_qwxyB, {c->qw_xyB.data(), c->qw_xyB.size() * sizeof(float2)}},
                {c->off_qwcoff, {c->qw_coff.data(), c->qw_coff.size() * 4}},
                {c->off_qwcorner, {c->qw_corner.data(), c->qw_corner.size() * sizeof(double2)}},
                {c->off_patch8, {c->patch8.data(), c->patch8.size() * 4}},
                {c->off_dgr, {c->q9_dgr.data(), c->q9_dgr.size() * sizeof(float2)}},
                {c->off_eflag, {c->q9_eflag.data(), c->q9_eflag.size()}}};
            for (const auto &u : up)
                if (u.second.second)
                    HIP_TRY(c, hipMemcpyAsync(c->ws + u.first, u.second.first, u.second.second,
                                              hipMemcpyHostToDevice, c->stream));
        }
        P.u_nblk = c->bh_off.empty() ? 0 : (int)c->bh_off.size() - 1;
        P.u_hmax = c->u_hmax;
        P.u_lemax = c->u_lemax;
        P.u_eu16 = c->u_eu16;
        if (!c->bh_off.empty()) {
            P.bh_off = reinterpret_cast<const int *>(c->ws + c->off_bh_off);
            P.bh_nodes = reinterpret_cast<const int *>(c->ws + c->off_bh_nodes);
            P.be_off = reinterpret_cast<const int *>(c->ws + c->off_be_off);
            P.be_elem = reinterpret_cast<const int *>(c->ws + c->off_be_elem);
            P.be_nodes = reinterpret_cast<const uint16_t *>(c->ws + c->off_be_nodes);
            P.uself = reinterpret_cast<const uint16_t *>(c->ws + c->off_uself);
            P.dep_le = reinterpret_cast<uint16_t *>(c->ws + c->off_dep_le);
            const std::pair<size_t, const void *> up[] = {
                {c->off_bh_off, c->bh_off.data()}, {c->off_bh_nodes, c->bh_nodes.data()},
                {c->off_be_off, c->be_off.data()}, {c->off_be_elem, c->be_elem.data()}};
            const size_t nbytes[] = {c->bh_off.size() * 4, c->bh_nodes.size() * 4, c->be_off.size() * 4,
                                     c->be_elem.size() * 4};
            for (int q = 0; q < 4; ++q)
                HIP_TRY(c, hipMemcpyAsync(c->ws + up[q].first, up[q].second, nbytes[q], hipMemcpyHostToDevice,
                                          c->stream));
            HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_be_nodes, c->be_nodes.data(), c->be_nodes.size() * 2,
                                      hipMemcpyHostToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_uself, c->uself.data(), c->uself.size() * 2,
                                      hipMemcpyHostToDevice, c->stream));
        } else {
            P.bh_off = P.bh_nodes = P.be_off = P.be_elem = nullptr;
            P.be_nodes = P.uself = nullptr;
            P.dep_le = nullptr;
        }
    }
    P.step = reinterpret_cast<long long *>(c->ws + c->off_step);
    P.err = reinterpret_cast<unsigned *>(c->ws + c->off_err);
    P.scratch = nullptr;
    const size_t N = (size_t)c->ni * c->nj;
    HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_X, c->X.data(), N * 16, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->ws + c->off_mask, 0, c->ni * 4, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->ws + c->off_force, 0, c->ni * 32, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->ws + c->off_hist, 0, (size_t)fsi::MAX_BODIES * fsi::HIST_CAP * 48,
                              c->stream));
    HIP_TRY(c, hipMemsetAsync(c->ws + c->off_step, 0, 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->ws + c->off_err, 0, 4, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->ws + c->off_resid, 0, fsi::MAX_BODIES * sizeof(double), c->stream));
    if (!c->wk0.empty()) {
        HIP_TRY(c, hipMemsetAsync(c->ws + c->off_cut, 0, (size_t)18 * c->inst.cut_n * 4, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_wk0, c->wk0.data(), c->wk0.size() * sizeof(int2),
                                  hipMemcpyHostToDevice, c->stream));
    }
    if (c->has_wall) {
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_B, c->wallB.data(), c->ni * 8, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_inflow, c->inflow.data(), c->inflow.size(),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_ff, c->ff.data(), c->ff.size() * sizeof(int2),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_wbnd, c->wbnd.data(), c->wbnd.size() * sizeof(int2),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_wwall, c->wwall.data(), c->wwall.size() * sizeof(int2),
                                  hipMemcpyHostToDevice, c->stream));
    }
    HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_wk1, c->wk1.data(), c->wk1.size() * sizeof(int2),
                              hipMemcpyHostToDevice, c->stream));
    if (!c->wk1s.empty())
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_wk1s, c->wk1s.data(), c->wk1s.size() * sizeof(int2),
                                  hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_inst, &c->inst, sizeof(Inst), hipMemcpyHostToDevice, c->stream));
    {
        fsi_status sn = upload_inst_na(c);
        if (sn != FSI_OK) return sn;
    }
    // static unstructured mesh: the departure points once
    if (c->topo == FSI_TOPO_Q9)
        HIP_TRY(c, fsi::launch_unstructured_locate(d_inst(c), (long long)c->ni, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->topo == FSI_TOPO_Q9) {
        unsigned e = 0;
        HIP_TRY(c, hipMemcpy(&e, c->ws + c->off_err, 4, hipMemcpyDeviceToHost));
        if (e & fsi::ERR_CFL)
            return fail(c, FSI_E_CFL, "a departure point lies outside the elements of its node "
                                      "(dt too large for this mesh)");
    }
    return FSI_OK;
}

fsi_status fsi_init_equilibrium(fsi_ctx *c, const double *rho, const double *ux, const double *uy,
                                const double *T) {
    fsi_status st = check_ready(c, false);
    if (st != FSI_OK) return st;
    const size_t N = (size_t)c->ni * c->nj;
    std::vector<double> macro(4 * N);
    const double dflt[4] = {c->fluid.rho_inf, c->fluid.u_inf[0], c->fluid.u_inf[1], c->fluid.T_inf};
    const double *src[4] = {rho, ux, uy, T};
    for (int k = 0; k < 4; ++k)
        for (size_t i = 0; i < N; ++i) macro[k * N + i] = src[k] ? src[k][i] : dflt[k];
    for (size_t i = 0; i < N; ++i) {
        const double r = macro[i], u = macro[N + i], v = macro[2 * N + i], t = macro[3 * N + i];
        if (!(r > 0) || !(t > 0) || !(1 - t - u * u > 0) || !(1 - t - v * v > 0))
            return fail(c, FSI_E_STATE, "initial state outside the D2Q9 positivity domain at node " +
                                            std::to_string(i));
    }
    double *scratch = reinterpret_cast<double *>(c->ws + c->off_pop[1]);
    HIP_TRY(c, hipMemcpyAsync(scratch, macro.data(), 4 * N * 8, hipMemcpyHostToDevice, c->stream));
    fsi::BodySlot slots[3][fsi::MAX_BODIES];
    for (int k = 0; k < fsi::MAX_BODIES; ++k) {
        slots[0][k] = slot_of(0, 0, 0, 0);
        if (k >= (int)c->bodies.size()) continue;
        // a linked body starts in the state of the body it moves with
        const int m = c->bodies[k].link >= 0 ? c->bodies[k].link : k;
        const fsi_body_desc &b = c->bodies[m];
        const bool forced = (b.dof == FSI_DOF_HEAVE || b.dof == FSI_DOF_PITCH_PLUNGE) && b.release_time > 0;
        if (b.dof == FSI_DOF_PRESCRIBED || forced)
            slots[0][k] = slot_of(0.0, 0.0, b.heave_amp * 2 * M_PI * b.heave_freq,
                                  b.pitch_amp * 2 * M_PI * b.pitch_freq);
        else
            slots[0][k] = slot_of(b.h0, b.a0, b.hd0, b.ad0);
    }
    for (int k = 0; k < fsi::MAX_BODIES; ++k) slots[1][k] = slots[2][k] = slots[0][k];
    HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_slots, slots, sizeof(slots), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->ws + c->off_step, 0, 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->ws + c->off_err, 0, 4, c->stream));
    HIP_TRY(c, fsi::launch_init_equilibrium(d_inst(c), scratch, (long long)N, c->fluid.storage, c->stream));
    st = enqueue_load_update(c);
    if (st != FSI_OK) return st;
    c->host_step = 0;
    c->initialized = true;
    return sync_check(c);
}

fsi_status fsi_step(fsi_ctx *c, int nsteps) {
    fsi_status st = check_ready(c, true);
    if (st != FSI_OK) return st;
    if (nsteps < 0) return fail(c, FSI_E_ARG, "nsteps < 0");
    if (nsteps == 0) return FSI_OK;
    if (c->stream == nullptr) {
        // the legacy default stream cannot be captured: launch directly
        for (int k = 0; k < nsteps; ++k) {
            st = enqueue_step(c);
            if (st != FSI_OK) return st;
        }
    } else {
        if (c->split && !c->stream2) {
            // the second stream of the split step (default priority), once
            HIP_TRY(c, hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking));
            HIP_TRY(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
            HIP_TRY(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
        }
        const int nlong = nsteps / kGraphSteps, nshort = nsteps % kGraphSteps;
        if (nlong && !c->graph_exec[1]) {
            st = capture_steps(c, 1, kGraphSteps);
            if (st != FSI_OK) return st;
        }
        if (nshort && !c->graph_exec[0]) {
            st = capture_steps(c, 0, 1);
            if (st != FSI_OK) return st;
        }
        for (int k = 0; k < nlong; ++k) HIP_TRY(c, hipGraphLaunch(c->graph_exec[1], c->stream));
        for (int k = 0; k < nshort; ++k) HIP_TRY(c, hipGraphLaunch(c->graph_exec[0], c->stream));
    }
    c->host_step += nsteps;
    return FSI_OK;
}

fsi_status fsi_step_noalloc(fsi_ctx *c, int nsteps) {
    fsi_status st = check_ready(c, true);
    if (st != FSI_OK) return st;
    if (nsteps < 0) return fail(c, FSI_E_ARG, "nsteps < 0");
    if (c->topo == FSI_TOPO_Q9) return fail(c, FSI_E_ARG, "fsi_step_noalloc: structured meshes only");
    if (!c->na_ready) {
        size_t off[5];
        return fail(c, FSI_E_ARG, "fsi_step_noalloc: the step needs " + std::to_string(na_layout(c, off)) +
                                      " bytes of scratch, more than the " +
                                      std::to_string(kNoAllocScratchBytes) + " the library holds");
    }
    // the kernels of each step, launched directly (no graph, no memset): the
    // same kernels as fsi_step with the per-step scratch in the static array;
    // every scratch entry a step reads is written earlier in the same step, so
    // nothing has to be cleared between calls
    for (int k = 0; k < nsteps; ++k) {
        st = enqueue_step(c, d_inst_na(c));
        if (st != FSI_OK) return st;
    }
    c->host_step += nsteps;
    return FSI_OK;
}

fsi_status fsi_synchronize(fsi_ctx *c) {
    fsi_status st = check_ready(c, false);
    if (st != FSI_OK) return st;
    return sync_check(c);
}

fsi_status fsi_get_step(fsi_ctx *c, int64_t *step) {
    fsi_status st = check_ready(c, true);
    if (st != FSI_OK) return st;
    if (!step) return fail(c, FSI_E_ARG, "null output");
    long long n = 0;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(&n, c->ws + c->off_step, 8, hipMemcpyDeviceToHost));
    *step = n;
    return FSI_OK;
}

fsi_status fsi_get_forces(fsi_ctx *c, int body, int64_t first, int count, double *out) {
    fsi_status st = check_ready(c, true);
    if (st != FSI_OK) return st;
    if (body < 0 || body >= std::max(1, (int)c->bodies.size()) || count < 0 || (count > 0 && !out))
        return fail(c, FSI_E_ARG, "bad history request");
    const int64_t last = c->host_step;   // record `last` exists once the queue drained
    const int64_t oldest = std::max<int64_t>(0, last - fsi::HIST_CAP + 1);
    if (first < oldest || first + count - 1 > last)
        return fail(c, FSI_E_ARG, "history records available: " + std::to_string(oldest) + " .. " +
                                      std::to_string(last));
    st = sync_check(c);
    if (st != FSI_OK) return st;
    for (int k = 0; k < count; ++k) {
        const int64_t L = first + k;
        HIP_TRY(c, hipMemcpy(out + 6 * (size_t)k,
                             c->ws + c->off_hist + ((size_t)body * fsi::HIST_CAP + (size_t)(L % fsi::HIST_CAP)) * 48,
                             48, hipMemcpyDeviceToHost));
    }
    return FSI_OK;
}

fsi_status fsi_get_body_state(fsi_ctx *c, int body, double out[4]) {
    fsi_status st = check_ready(c, true);
    if (st != FSI_OK) return st;
    if (body < 0 || body >= std::max(1, (int)c->bodies.size()) || !out)
        return fail(c, FSI_E_ARG, "bad body index");
    st = sync_check(c);
    if (st != FSI_OK) return st;
    fsi::BodySlot s;
    HIP_TRY(c, hipMemcpy(&s, c->ws + c->off_slots +
                                 ((size_t)(c->host_step % 3) * fsi::MAX_BODIES + body) * sizeof(fsi::BodySlot),
                         sizeof(s), hipMemcpyDeviceToHost));
    out[0] = s.h; out[1] = s.a; out[2] = s.hd; out[3] = s.ad;
    return FSI_OK;
}

fsi_status fsi_dump_macro(fsi_ctx *c, double *rho, double *ux, double *uy, double *T) {
    fsi_status st = check_ready(c, true);
    if (st != FSI_OK) return st;
    const size_t N = (size_t)c->ni * c->nj;
    const int cur = (int)(c->host_step & 1);
    double *scratch = reinterpret_cast<double *>(c->ws + c->off_pop[cur ^ 1]);
    HIP_TRY(c, fsi::launch_dump_macro(d_inst(c), cur, scratch, (long long)N, c->fluid.storage, c->stream));
    st = sync_check(c);
    if (st != FSI_OK) return st;
    double *outs[4] = {rho, ux, uy, T};
    for (int k = 0; k < 4; ++k)
        if (outs[k]) HIP_TRY(c, hipMemcpy(outs[k], scratch + k * N, N * 8, hipMemcpyDeviceToHost));
    return FSI_OK;
}

fsi_status fsi_get_populations(fsi_ctx *c, float *f, float *g) {
    fsi_status st = check_ready(c, true);
    if (st != FSI_OK) return st;
    const size_t N = (size_t)c->ni * c->nj;
    const int cur = (int)(c->host_step & 1);
    st = sync_check(c);
    if (st != FSI_OK) return st;
    float *outs[2] = {f, g};
    for (int h = 0; h < 2; ++h) {
        if (!outs[h]) continue;
        if (c->fluid.storage == FSI_STORE_FP32) {
            HIP_TRY(c, hipMemcpy(outs[h], c->ws + c->off_pop[cur] + (size_t)h * 9 * N * 4, 9 * N * 4,
                                 hipMemcpyDeviceToHost));
        } else {
            float *tmp = reinterpret_cast<float *>(c->ws + c->off_pop[cur ^ 1]);
            HIP_TRY(c, fsi::launch_decode(d_inst(c), cur, 9 * h, tmp, (long long)N, 1, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            HIP_TRY(c, hipMemcpy(outs[h], tmp, 9 * N * 4, hipMemcpyDeviceToHost));
        }
    }
    return FSI_OK;
}

fsi_status fsi_set_populations(fsi_ctx *c, const float *f, const float *g) {
    fsi_status st = check_ready(c, true);
    if (st != FSI_OK) return st;
    if (!f || !g) return fail(c, FSI_E_ARG, "null populations");
    const size_t N = (size_t)c->ni * c->nj;
    const int cur = (int)(c->host_step & 1);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const float *ins[2] = {f, g};
    for (int h = 0; h < 2; ++h) {
        if (c->fluid.storage == FSI_STORE_FP32) {
            HIP_TRY(c, hipMemcpy(c->ws + c->off_pop[cur] + (size_t)h * 9 * N * 4, ins[h], 9 * N * 4,
                                 hipMemcpyHostToDevice));
        } else {
            float *tmp = reinterpret_cast<float *>(c->ws + c->off_pop[cur ^ 1]);
            HIP_TRY(c, hipMemcpy(tmp, ins[h], 9 * N * 4, hipMemcpyHostToDevice));
            HIP_TRY(c, fsi::launch_encode(d_inst(c), cur, 9 * h, tmp, (long long)N, 1, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
        }
    }
    // the load of the new populations and the body state it drives
    st = enqueue_load_update(c);
    if (st != FSI_OK) return st;
    return sync_check(c);
}

fsi_status fsi_state_bytes(const fsi_ctx *c, size_t *bytes) {
    if (!c || !bytes) return FSI_E_ARG;
    const size_t N = (size_t)c->ni * c->nj;
    const size_t bpp = c->fluid.storage == FSI_STORE_FP16_SHIFTED ? 2 : 4;
    // a moving body on a Q9 mesh: the departure table (element, local
    // coordinates), from which each step's relocation starts
    const size_t dep = c->q9_moving ? 9 * N * (sizeof(int) + sizeof(float2)) : 0;
    *bytes = 8 * 6 + 3 * fsi::MAX_BODIES * sizeof(fsi::BodySlot) + fsi::NPOP * N * bpp + dep;
    return FSI_OK;
}

fsi_status fsi_save(fsi_ctx *c, void *host_buf, size_t bytes) {
    fsi_status st = check_ready(c, true);
    if (st != FSI_OK) return st;
    size_t need = 0;
    fsi_state_bytes(c, &need);
    if (!host_buf || bytes < need) return fail(c, FSI_E_ARG, "checkpoint buffer too small");
    st = sync_check(c);
    if (st != FSI_OK) return st;
    const size_t N = (size_t)c->ni * c->nj;
    const size_t bpp = c->fluid.storage == FSI_STORE_FP16_SHIFTED ? 2 : 4;
    int64_t *hdr = static_cast<int64_t *>(host_buf);
    hdr[0] = kMagic; hdr[1] = c->ni; hdr[2] = c->nj; hdr[3] = c->fluid.storage; hdr[4] = c->host_step;
    hdr[5] = c->topo;
    char *p = static_cast<char *>(host_buf) + 48;
    HIP_TRY(c, hipMemcpy(p, c->ws + c->off_slots, 3 * fsi::MAX_BODIES * sizeof(fsi::BodySlot),
                         hipMemcpyDeviceToHost));
    p += 3 * fsi::MAX_BODIES * sizeof(fsi::BodySlot);
    HIP_TRY(c, hipMemcpy(p, c->ws + c->off_pop[c->host_step & 1], fsi::NPOP * N * bpp, hipMemcpyDeviceToHost));
    p += fsi::NPOP * N * bpp;
    if (c->q9_moving) {
        HIP_TRY(c, hipMemcpy(p, c->ws + c->off_dep_e, 9 * N * sizeof(int), hipMemcpyDeviceToHost));
        p += 9 * N * sizeof(int);
        HIP_TRY(c, hipMemcpy(p, c->ws + c->off_dep_xy, 9 * N * sizeof(float2), hipMemcpyDeviceToHost));
    }
    return FSI_OK;
}

fsi_status fsi_load(fsi_ctx *c, const void *host_buf, size_t bytes) {
    fsi_status st = check_ready(c, false);
    if (st != FSI_OK) return st;
    size_t need = 0;
    fsi_state_bytes(c, &need);
    if (!host_buf || bytes < need) return fail(c, FSI_E_ARG, "checkpoint buffer too small");
    const int64_t *hdr = static_cast<const int64_t *>(host_buf);
    if (hdr[0] != kMagic || hdr[1] != c->ni || hdr[2] != c->nj || hdr[3] != c->fluid.storage || hdr[5] != c->topo)
        return fail(c, FSI_E_ARG, "checkpoint does not match this context");
    const size_t N = (size_t)c->ni * c->nj;
    const size_t bpp = c->fluid.storage == FSI_STORE_FP16_SHIFTED ? 2 : 4;
    const int64_t step = hdr[4];
    const char *p = static_cast<const char *>(host_buf) + 48;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(c->ws + c->off_slots, p, 3 * fsi::MAX_BODIES * sizeof(fsi::BodySlot),
                         hipMemcpyHostToDevice));
    p += 3 * fsi::MAX_BODIES * sizeof(fsi::BodySlot);
    HIP_TRY(c, hipMemcpy(c->ws + c->off_pop[step & 1], p, fsi::NPOP * N * bpp, hipMemcpyHostToDevice));
    p += fsi::NPOP * N * bpp;
    if (c->q9_moving) {
        // the departure table the run continues from: elements and local
        // coordinates (element ids checked on the host), then the block-list
        // positions formed from them
        std::vector<int> de(9 * N);
        memcpy(de.data(), p, 9 * N * sizeof(int));
        for (size_t q = 0; q < de.size(); ++q) {
            // -1 missing; -2 (the rest plane only) the node itself
            const int lo = q >= 8 * N ? -2 : -1;
            if (de[q] < lo || de[q] >= c->n_elems) return fail(c, FSI_E_ARG, "checkpoint departure table out of range");
        }
        HIP_TRY(c, hipMemcpy(c->ws + c->off_dep_e, de.data(), 9 * N * sizeof(int), hipMemcpyHostToDevice));
        p += 9 * N * sizeof(int);
        HIP_TRY(c, hipMemcpy(c->ws + c->off_dep_xy, p, 9 * N * sizeof(float2), hipMemcpyHostToDevice));
        if (!c->bh_off.empty())
            HIP_TRY(c, fsi::launch_unstructured_dep_le(d_inst(c), (long long)N, c->stream));
    }
    long long s = step;
    HIP_TRY(c, hipMemcpy(c->ws + c->off_step, &s, 8, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemset(c->ws + c->off_err, 0, 4));
    c->host_step = step;
    c->initialized = true;
    // the history record of the current level
    st = enqueue_load_update(c);
    if (st != FSI_OK) return st;
    return sync_check(c);
}

fsi_status fsi_time_kernels(fsi_ctx *c, int reps, double out_ms[4]) {
    fsi_status st = check_ready(c, true);
    if (st != FSI_OK) return st;
    if (reps < 1 || !out_ms) return fail(c, FSI_E_ARG, "reps must be >= 1");
    st = sync_check(c);
    if (st != FSI_OK) return st;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    const int stg = c->fluid.storage;
    const int2 *wk1 = reinterpret_cast<const int2 *>(c->ws + c->off_wk1);
    const int2 *wbnd = reinterpret_cast<const int2 *>(c->ws + c->off_wbnd);
    const int2 *wwall = reinterpret_cast<const int2 *>(c->ws + c->off_wwall);
    for (int which = 0; which < 4; ++which) {
        out_ms[which] = 0.0;
        if (!c->has_wall && (which == 1 || which == 2)) continue;
        // one untimed launch, then `reps` timed ones
        for (int r = 0; r <= reps; ++r) {
            if (r == 1) HIP_TRY(c, hipEventRecord(e0, c->stream));
            hipError_t e = hipSuccess;
            if (which == 0 && !c->wk0.empty())
                HIP_TRY(c, fsi::launch_cut_export(d_inst(c), reinterpret_cast<const int2 *>(c->ws + c->off_wk0),
                                                  (int)c->wk0.size(), stg, c->stream));
            if (which == 0 && c->topo == FSI_TOPO_Q9)
                e = fsi::launch_unstructured(d_inst(c), (long long)c->ni, (long long)c->n_elems, stg,
                                             c->inst.uq, c->inst.ud, c->inst.ueg, c->inst.u_nblk,
                                             c->inst.u_hmax, c->inst.u_lemax, c->inst.u_eu16, c->inst.qdisp,
                                             0, c->stream);
            else if (which == 0)
                e = fsi::launch_collide_stream(d_inst(c), wk1, (int)c->wk1.size(), stg, c->stream, 0,
                                               c->cut, c->shape, c->stream_out);
            if (which == 1) e = fsi::launch_wall_targets(d_inst(c), wbnd, (int)c->wbnd.size(), stg, c->stream);
            // phase 0 of the wall kernel (traction only) and of the body kernel
            // recompute the current level without advancing it
            if (which == 2) e = fsi::launch_wall_grad_force(d_inst(c), wwall, (int)c->wwall.size(), stg, 0, c->stream);
            if (which == 3) e = fsi::launch_body(d_inst(c), 1, 0, c->stream);
            HIP_TRY(c, e);
        }
        HIP_TRY(c, hipEventRecord(e1, c->stream));
        HIP_TRY(c, hipEventSynchronize(e1));
        float ms = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
        out_ms[which] = ms / reps;
    }
    HIP_TRY(c, hipEventDestroy(e0));
    HIP_TRY(c, hipEventDestroy(e1));
    // the repeated unstructured launches left the moments of the scratch side
    if (c->topo == FSI_TOPO_Q9)
        HIP_TRY(c, fsi::launch_unstructured_moments(d_inst(c), (long long)c->ni, c->fluid.storage, c->stream));
    return sync_check(c);
}

fsi_status fsi_set_coupling(fsi_ctx *c, int subiterations, double relaxation) {
    if (!c) return FSI_E_ARG;
    if (subiterations < 1 || subiterations > 64 || !(relaxation > 0.0 && relaxation <= 1.0))
        return fail(c, FSI_E_ARG, "coupling needs 1 <= subiterations <= 64 and 0 < relaxation <= 1");
    drop_graph(c);
    c->n_sub = subiterations;
    c->relax = relaxation;
    c->inst.n_sub = subiterations;
    c->inst.relax = relaxation;
    if (c->ws) {
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_inst, &c->inst, sizeof(Inst), hipMemcpyHostToDevice,
                                  c->stream));
        fsi_status sn = upload_inst_na(c);
        if (sn != FSI_OK) return sn;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return FSI_OK;
}

fsi_status fsi_get_coupling_residual(fsi_ctx *c, int body, double *residual) {
    fsi_status st = check_ready(c, true);
    if (st != FSI_OK) return st;
    if (body < 0 || body >= std::max(1, (int)c->bodies.size()) || !residual)
        return fail(c, FSI_E_ARG, "bad body index");
    st = sync_check(c);
    if (st != FSI_OK) return st;
    HIP_TRY(c, hipMemcpy(residual, c->ws + c->off_resid + (size_t)body * sizeof(double), sizeof(double),
                         hipMemcpyDeviceToHost));
    return FSI_OK;
}

const char *fsi_last_error(const fsi_ctx *c) { return c ? c->err.c_str() : "null context"; }

void fsi_destroy(fsi_ctx *c) {
    if (!c) return;
    // the caller frees the workspace after this returns: drain queued work first
    if (c->ws) (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    if (c->stream2) {
        (void)hipStreamSynchronize(c->stream2);
        (void)hipStreamDestroy(c->stream2);
        (void)hipEventDestroy(c->ev_fork);
        (void)hipEventDestroy(c->ev_join);
    }
    delete c;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches of independent instances
// ---------------------------------------------------------------------------
struct fsi_batch {
    std::vector<fsi_ctx *> ctx;
    hipStream_t stream = nullptr;
    int storage = 0;
    bool any_wall = false;
    size_t off_insts = 0, off_wk0 = 0, off_wk1 = 0, off_wbnd = 0, off_wwall = 0, total = 0;
    std::vector<size_t> off_region;
    char *ws = nullptr;
    std::vector<int2> wk0, wk1, wbnd, wwall;
    int grid = 0, order = 0, shape = 0;
    int n_sub = 1;                  // coupling sub-iterations per step (all instances)
    bool any_cut = false;           // an instance needs the cut build (a cut or two bodies)
    bool any_plain = false;         // an instance does not
    int n_cut_items = 0;            // wk1 holds these instances' 32 x 16 tiles first
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    std::string err;
};

namespace {

fsi_status bfail(fsi_batch *b, fsi_status st, const std::string &msg) {
    if (b) b->err = msg;
    return st;
}

#define BHIP_TRY(b, expr)                                                            \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) return bfail(b, FSI_E_HIP, std::string(#expr) + ": " + \
                                                         hipGetErrorString(e_));     \
    } while (0)

void batch_drop_graph(fsi_batch *b) {
    for (int q = 0; q < 2; ++q) {
        if (b->graph_exec[q]) (void)hipGraphExecDestroy(b->graph_exec[q]);
        if (b->graph[q]) (void)hipGraphDestroy(b->graph[q]);
        b->graph_exec[q] = nullptr;
        b->graph[q] = nullptr;
    }
}

// instances the fused kernel's cut build serves (a cut, or two bodies)
bool needs_cut_build(const fsi_ctx *c) { return c->cut || c->bodies.size() > 1; }

void batch_lists(fsi_batch *b) {
    const int n = (int)b->ctx.size();
    std::vector<int> ord(n);
    for (int k = 0; k < n; ++k) ord[k] = k;
    if (b->order == 1)
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) {
            return b->ctx[a]->inst.n_nodes > b->ctx[c]->inst.n_nodes;
        });
    b->wk0.clear();
    b->wk1.clear();
    b->wbnd.clear();
    b->wwall.clear();
    // instances that need the cut build run on 32 x 16 tiles (the only shape
    // of that build), the others on the scheduled shape; each instance's
    // tiles in row order (an XCD's run of the list spans several instances)
    for (int pass = 0; pass < 2; ++pass) {
        const int sh = pass == 0 ? 0 : b->shape;
        for (int k : ord) {
            const fsi_ctx *c = b->ctx[k];
            if (needs_cut_build(c) != (pass == 0)) continue;
            append_tiles(b->wk1, k, c->ni, c->nj, sh, 1);
        }
        if (pass == 0) b->n_cut_items = (int)b->wk1.size();
    }
    // the per-instance lists, re-labelled with the instance index
    for (int k = 0; k < n; ++k) {
        for (int2 w : b->ctx[k]->wk0) b->wk0.push_back(make_int2(k, w.y));
        for (int2 w : b->ctx[k]->wbnd) b->wbnd.push_back(make_int2(k, w.y));
        for (int2 w : b->ctx[k]->wwall) b->wwall.push_back(make_int2(k, w.y));
    }
}

fsi_status batch_upload_lists(fsi_batch *b) {
    if (!b->wk0.empty())
        BHIP_TRY(b, hipMemcpyAsync(b->ws + b->off_wk0, b->wk0.data(), b->wk0.size() * sizeof(int2),
                                   hipMemcpyHostToDevice, b->stream));
    BHIP_TRY(b, hipMemcpyAsync(b->ws + b->off_wk1, b->wk1.data(), b->wk1.size() * sizeof(int2),
                               hipMemcpyHostToDevice, b->stream));
    if (!b->wbnd.empty()) {
        BHIP_TRY(b, hipMemcpyAsync(b->ws + b->off_wbnd, b->wbnd.data(), b->wbnd.size() * sizeof(int2),
                                   hipMemcpyHostToDevice, b->stream));
        BHIP_TRY(b, hipMemcpyAsync(b->ws + b->off_wwall, b->wwall.data(), b->wwall.size() * sizeof(int2),
                                   hipMemcpyHostToDevice, b->stream));
    }
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    return FSI_OK;
}

const Inst *b_insts(fsi_batch *b) { return reinterpret_cast<const Inst *>(b->ws + b->off_insts); }

fsi_status batch_enqueue_k1(fsi_batch *b) {
    if (!b->wk0.empty())
        BHIP_TRY(b, fsi::launch_cut_export(b_insts(b), reinterpret_cast<const int2 *>(b->ws + b->off_wk0),
                                           (int)b->wk0.size(), b->storage, b->stream));
    const int2 *wk1 = reinterpret_cast<const int2 *>(b->ws + b->off_wk1);
    const int n_plain = (int)b->wk1.size() - b->n_cut_items;
    if (b->n_cut_items > 0)
        BHIP_TRY(b, fsi::launch_collide_stream(b_insts(b), wk1, b->n_cut_items, b->storage, b->stream,
                                               b->grid, true, 0));
    if (n_plain > 0)
        BHIP_TRY(b, fsi::launch_collide_stream(b_insts(b), wk1 + b->n_cut_items, n_plain, b->storage,
                                               b->stream, b->grid, false, b->shape));
    return FSI_OK;
}

fsi_status batch_enqueue_step(fsi_batch *b) {
    for (int k = 0; k < b->n_sub; ++k) {
        fsi_status st = batch_enqueue_k1(b);
        if (st != FSI_OK) return st;
        if (b->any_wall) {
            BHIP_TRY(b, fsi::launch_wall_targets(b_insts(b), reinterpret_cast<const int2 *>(b->ws + b->off_wbnd),
                                                 (int)b->wbnd.size(), b->storage, b->stream));
            BHIP_TRY(b, fsi::launch_wall_grad_force(b_insts(b),
                                                    reinterpret_cast<const int2 *>(b->ws + b->off_wwall),
                                                    (int)b->wwall.size(), b->storage, 1, b->stream));
        }
        BHIP_TRY(b, fsi::launch_body(b_insts(b), (int)b->ctx.size(), k + 1 < b->n_sub ? 2 : 1, b->stream));
    }
    return FSI_OK;
}

fsi_status batch_ready(fsi_batch *b, int k) {
    if (!b) return FSI_E_ARG;
    if (!b->ws) return bfail(b, FSI_E_UNBOUND, "workspace not bound");
    if (k >= (int)b->ctx.size()) return bfail(b, FSI_E_ARG, "no such instance");
    if (k < 0)
        for (fsi_ctx *c : b->ctx)
            if (!c->initialized) return bfail(b, FSI_E_UNBOUND, "an instance is not initialised");
    return FSI_OK;
}

// forward a per-instance status and message
fsi_status bfwd(fsi_batch *b, int k, fsi_status st) {
    if (st != FSI_OK) b->err = "instance " + std::to_string(k) + ": " + b->ctx[k]->err;
    return st;
}

}  // namespace

extern "C" {

fsi_status fsi_batch_create(int n, const fsi_fluid_params *fluids, const fsi_mesh_desc *meshes,
                            const fsi_body_desc *bodies, const int *nbodies, void *hip_stream,
                            fsi_batch **out) {
    if (!out) return FSI_E_ARG;
    *out = nullptr;
    fsi_batch *b = new (std::nothrow) fsi_batch();
    if (!b) return FSI_E_NOMEM;
    *out = b;
    if (n < 1 || !fluids || !meshes) return bfail(b, FSI_E_ARG, "need n >= 1 fluids and meshes");
    b->stream = (hipStream_t)hip_stream;
    size_t first_body = 0;
    for (int k = 0; k < n; ++k) {
        const int nb = nbodies ? nbodies[k] : 0;
        if (nb && !bodies) return bfail(b, FSI_E_ARG, "bodies missing");
        if (nb < 0) return bfail(b, FSI_E_ARG, "instance " + std::to_string(k) + ": nbodies < 0");
        fsi_ctx *c = nullptr;
        const fsi_status st = fsi_create(&fluids[k], &meshes[k], nb ? &bodies[first_body] : nullptr, nb,
                                         hip_stream, &c);
        first_body += (size_t)nb;
        if (st != FSI_OK) {
            b->err = "instance " + std::to_string(k) + ": " + (c ? c->err : std::string("create failed"));
            fsi_destroy(c);
            return st;
        }
        b->ctx.push_back(c);
        if (c->topo == FSI_TOPO_Q9)
            return bfail(b, FSI_E_ARG, "instance " + std::to_string(k) + ": Q9 meshes run as single contexts");
        if (k == 0) b->storage = c->fluid.storage;
        if (c->fluid.storage != b->storage) return bfail(b, FSI_E_ARG, "mixed storage precisions");
        if (c->has_wall) b->any_wall = true;
        if (needs_cut_build(c)) b->any_cut = true;
        else b->any_plain = true;
    }
    // the default of the instances without a cut (those with one always use
    // 32 x 16): 32 x 16 too; the autotuner picks the fastest
    batch_lists(b);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + std::max<size_t>(bytes, 1)); return r; };
    b->off_insts = take(n * sizeof(Inst));
    b->off_wk0 = take(b->wk0.size() * sizeof(int2));
    size_t max_items = 0;                 // the largest work list over the shapes
    for (int sh = 0; sh < fsi::N_TILE_SHAPES; ++sh) {
        size_t items = 0;
        for (fsi_ctx *c : b->ctx) {
            const int s2 = needs_cut_build(c) ? 0 : sh;
            const int tx = fsi::TILE_SHAPES[s2][0], ty = fsi::TILE_SHAPES[s2][1];
            items += (size_t)((c->ni + tx - 1) / tx) * ((c->nj + ty - 1) / ty);
        }
        max_items = std::max(max_items, items);
    }
    b->off_wk1 = take(max_items * sizeof(int2));
    b->off_wbnd = take(b->wbnd.size() * sizeof(int2));
    b->off_wwall = take(b->wwall.size() * sizeof(int2));
    for (fsi_ctx *c : b->ctx) b->off_region.push_back(take(c->total));
    b->total = o;
    return FSI_OK;
}

fsi_status fsi_batch_workspace_bytes(const fsi_batch *b, size_t *bytes) {
    if (!b || !bytes) return FSI_E_ARG;
    *bytes = b->total;
    return FSI_OK;
}

fsi_status fsi_batch_bind_workspace(fsi_batch *b, void *dev_ptr, size_t bytes) {
    if (!b || !dev_ptr) return FSI_E_ARG;
    if (((uintptr_t)dev_ptr & 255) != 0) return bfail(b, FSI_E_ARG, "workspace must be 256-byte aligned");
    if (bytes < b->total) return bfail(b, FSI_E_ARG, "workspace too small");
    batch_drop_graph(b);
    b->ws = static_cast<char *>(dev_ptr);
    std::vector<Inst> insts(b->ctx.size());
    for (size_t k = 0; k < b->ctx.size(); ++k) {
        fsi_status st = fsi_bind_workspace(b->ctx[k], b->ws + b->off_region[k], b->ctx[k]->total);
        if (st != FSI_OK) return bfwd(b, (int)k, st);
        insts[k] = b->ctx[k]->inst;
    }
    BHIP_TRY(b, hipMemcpyAsync(b->ws + b->off_insts, insts.data(), insts.size() * sizeof(Inst),
                               hipMemcpyHostToDevice, b->stream));
    return batch_upload_lists(b);
}

fsi_status fsi_batch_init_equilibrium(fsi_batch *b, int k, const double *rho, const double *ux,
                                      const double *uy, const double *T) {
    fsi_status st = batch_ready(b, k);
    if (st != FSI_OK) return st;
    if (k < 0) return bfail(b, FSI_E_ARG, "no such instance");
    return bfwd(b, k, fsi_init_equilibrium(b->ctx[k], rho, ux, uy, T));
}

fsi_status fsi_batch_set_schedule(fsi_batch *b, int grid, int order, int shape) {
    if (!b) return FSI_E_ARG;
    if (grid < 0 || (order != 0 && order != 1) || shape < 0 || shape >= fsi::N_TILE_SHAPES)
        return bfail(b, FSI_E_ARG, "bad schedule");
    batch_drop_graph(b);
    b->grid = grid;
    if (order != b->order || shape != b->shape) {
        b->order = order;
        b->shape = shape;
        batch_lists(b);
        if (b->ws) return batch_upload_lists(b);
    }
    return FSI_OK;
}

fsi_status fsi_batch_step(fsi_batch *b, int nsteps) {
    fsi_status st = batch_ready(b, -1);
    if (st != FSI_OK) return st;
    if (nsteps < 0) return bfail(b, FSI_E_ARG, "nsteps < 0");
    if (nsteps == 0) return FSI_OK;
    if (b->stream == nullptr) {
        for (int k = 0; k < nsteps; ++k) {
            st = batch_enqueue_step(b);
            if (st != FSI_OK) return st;
        }
    } else {
        const int nlong = nsteps / kGraphSteps, nshort = nsteps % kGraphSteps;
        for (int q = 0; q < 2; ++q) {
            if ((q ? nlong : nshort) == 0 || b->graph_exec[q]) continue;
            BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            st = FSI_OK;
            for (int k = 0; k < (q ? kGraphSteps : 1) && st == FSI_OK; ++k) st = batch_enqueue_step(b);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(b->stream, &g);
            if (st != FSI_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) return bfail(b, FSI_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            b->graph[q] = g;
            BHIP_TRY(b, hipGraphInstantiate(&b->graph_exec[q], g, nullptr, nullptr, 0));
        }
        for (int k = 0; k < nlong; ++k) BHIP_TRY(b, hipGraphLaunch(b->graph_exec[1], b->stream));
        for (int k = 0; k < nshort; ++k) BHIP_TRY(b, hipGraphLaunch(b->graph_exec[0], b->stream));
    }
    for (fsi_ctx *c : b->ctx) c->host_step += nsteps;
    return FSI_OK;
}

fsi_status fsi_batch_synchronize(fsi_batch *b) {
    fsi_status st = batch_ready(b, 0);
    if (st != FSI_OK) return st;
    for (size_t k = 0; k < b->ctx.size(); ++k) {
        st = fsi_synchronize(b->ctx[k]);
        if (st != FSI_OK) return bfwd(b, (int)k, st);
    }
    return FSI_OK;
}

fsi_status fsi_batch_get_forces(fsi_batch *b, int k, int body, int64_t first, int count,
                                double *out) {
    fsi_status st = batch_ready(b, k);
    if (st != FSI_OK) return st;
    if (k < 0) return bfail(b, FSI_E_ARG, "no such instance");
    return bfwd(b, k, fsi_get_forces(b->ctx[k], body, first, count, out));
}

fsi_status fsi_batch_get_body_state(fsi_batch *b, int k, int body, double out[4]) {
    fsi_status st = batch_ready(b, k);
    if (st != FSI_OK) return st;
    if (k < 0) return bfail(b, FSI_E_ARG, "no such instance");
    return bfwd(b, k, fsi_get_body_state(b->ctx[k], body, out));
}

fsi_status fsi_batch_dump_macro(fsi_batch *b, int k, double *rho, double *ux, double *uy, double *T) {
    fsi_status st = batch_ready(b, k);
    if (st != FSI_OK) return st;
    if (k < 0) return bfail(b, FSI_E_ARG, "no such instance");
    return bfwd(b, k, fsi_dump_macro(b->ctx[k], rho, ux, uy, T));
}

fsi_status fsi_batch_get_populations(fsi_batch *b, int k, float *f, float *g) {
    fsi_status st = batch_ready(b, k);
    if (st != FSI_OK) return st;
    if (k < 0) return bfail(b, FSI_E_ARG, "no such instance");
    return bfwd(b, k, fsi_get_populations(b->ctx[k], f, g));
}

fsi_status fsi_batch_time_kernels(fsi_batch *b, int reps, double out_ms[4]) {
    fsi_status st = batch_ready(b, -1);
    if (st != FSI_OK) return st;
    if (reps < 1 || !out_ms) return bfail(b, FSI_E_ARG, "reps must be >= 1");
    st = fsi_batch_synchronize(b);
    if (st != FSI_OK) return st;
    hipEvent_t e0, e1;
    BHIP_TRY(b, hipEventCreate(&e0));
    BHIP_TRY(b, hipEventCreate(&e1));
    const int2 *wbnd = reinterpret_cast<const int2 *>(b->ws + b->off_wbnd);
    const int2 *wwall = reinterpret_cast<const int2 *>(b->ws + b->off_wwall);
    for (int which = 0; which < 4; ++which) {
        out_ms[which] = 0.0;
        if (!b->any_wall && (which == 1 || which == 2)) continue;
        for (int r = 0; r <= reps; ++r) {
            if (r == 1) BHIP_TRY(b, hipEventRecord(e0, b->stream));
            if (which == 0) {
                st = batch_enqueue_k1(b);
                if (st != FSI_OK) return st;
            }
            if (which == 1) BHIP_TRY(b, fsi::launch_wall_targets(b_insts(b), wbnd, (int)b->wbnd.size(), b->storage, b->stream));
            if (which == 2) BHIP_TRY(b, fsi::launch_wall_grad_force(b_insts(b), wwall, (int)b->wwall.size(), b->storage, 0, b->stream));
            if (which == 3) BHIP_TRY(b, fsi::launch_body(b_insts(b), (int)b->ctx.size(), 0, b->stream));
        }
        BHIP_TRY(b, hipEventRecord(e1, b->stream));
        BHIP_TRY(b, hipEventSynchronize(e1));
        float ms = 0.0f;
        BHIP_TRY(b, hipEventElapsedTime(&ms, e0, e1));
        out_ms[which] = ms / reps;
    }
    BHIP_TRY(b, hipEventDestroy(e0));
    BHIP_TRY(b, hipEventDestroy(e1));
    return fsi_batch_synchronize(b);
}

fsi_status fsi_batch_autotune(fsi_batch *b, int reps, double best[4]) {
    fsi_status st = batch_ready(b, -1);
    if (st != FSI_OK) return st;
    if (reps < 1 || !best) return bfail(b, FSI_E_ARG, "reps must be >= 1");
    // candidate grids: one workgroup per item, and persistent grids of a few
    // multiples of the resident capacity (256 CUs x 2 tiles)
    const int grids[] = {0, 4096, 2048, 1024, 512};
    double best_ms = 1e30;
    int best_grid = 0, best_order = 0, best_shape = 0;
    const int n_shapes = b->any_plain ? fsi::N_TILE_SHAPES : 1;
    // warm-up launches first (clocks ramp up over the first milliseconds),
    // then each candidate timed twice and its faster pass kept
    {
        double ms[4];
        st = fsi_batch_time_kernels(b, 4 * reps + 8, ms);
        if (st != FSI_OK) return st;
    }
    for (int pass = 0; pass < 2; ++pass) {
        for (int shape = 0; shape < n_shapes; ++shape) {
            for (int order = 0; order <= 1; ++order) {
                for (int grid : grids) {
                    st = fsi_batch_set_schedule(b, grid, order, shape);
                    if (st != FSI_OK) return st;
                    double ms[4];
                    st = fsi_batch_time_kernels(b, reps, ms);
                    if (st != FSI_OK) return st;
                    if (ms[0] < best_ms) {
                        best_ms = ms[0];
                        best_grid = grid;
                        best_order = order;
                        best_shape = shape;
                    }
                }
            }
        }
    }
    st = fsi_batch_set_schedule(b, best_grid, best_order, best_shape);
    if (st != FSI_OK) return st;
    best[0] = best_grid;
    best[1] = best_order;
    best[2] = best_shape;
    best[3] = best_ms;
    return FSI_OK;
}

fsi_status fsi_batch_set_coupling(fsi_batch *b, int subiterations, double relaxation) {
    if (!b) return FSI_E_ARG;
    for (size_t k = 0; k < b->ctx.size(); ++k) {
        fsi_ctx *c = b->ctx[k];
        if (subiterations < 1 || subiterations > 64 || !(relaxation > 0.0 && relaxation <= 1.0))
            return bfail(b, FSI_E_ARG, "coupling needs 1 <= subiterations <= 64 and 0 < relaxation <= 1");
        c->n_sub = subiterations;
        c->relax = relaxation;
        c->inst.n_sub = subiterations;
        c->inst.relax = relaxation;
    }
    batch_drop_graph(b);
    b->n_sub = subiterations;
    if (b->ws) {
        std::vector<Inst> insts(b->ctx.size());
        for (size_t k = 0; k < b->ctx.size(); ++k) {
            insts[k] = b->ctx[k]->inst;
            BHIP_TRY(b, hipMemcpyAsync(b->ctx[k]->ws + b->ctx[k]->off_inst, &b->ctx[k]->inst, sizeof(Inst),
                                       hipMemcpyHostToDevice, b->stream));
        }
        BHIP_TRY(b, hipMemcpyAsync(b->ws + b->off_insts, insts.data(), insts.size() * sizeof(Inst),
                                   hipMemcpyHostToDevice, b->stream));
        BHIP_TRY(b, hipStreamSynchronize(b->stream));
    }
    return FSI_OK;
}

int64_t fsi_batch_nodes(const fsi_batch *b) {
    int64_t n = 0;
    if (b)
        for (const fsi_ctx *c : b->ctx) n += (int64_t)c->ni * c->nj;
    return n;
}

const char *fsi_batch_last_error(const fsi_batch *b) { return b ? b->err.c_str() : "null batch"; }

void fsi_batch_destroy(fsi_batch *b) {
    if (!b) return;
    if (b->ws) (void)hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    for (fsi_ctx *c : b->ctx) fsi_destroy(c);
    delete b;
}

}  // extern "C"
