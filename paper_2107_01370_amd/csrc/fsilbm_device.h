// Device code shared by the structured-mesh kernels and the unstructured
// 9-node element kernels: population storage accessors, blending and rigid
// maps, moments, equilibria and the collision (Sec. II.C, II.D).  Included by
// the kernel sources only.
#pragma once

#include "fsilbm_internal.h"

namespace fsi {

#define CXK(k) ((k) == 1 || (k) == 5 || (k) == 8 ? 1 : ((k) == 3 || (k) == 6 || (k) == 7 ? -1 : 0))
#define CYK(k) ((k) == 2 || (k) == 5 || (k) == 6 ? 1 : ((k) == 4 || (k) == 7 || (k) == 8 ? -1 : 0))

__device__ __forceinline__ int floor_div(int a, int b) {
    const int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}
__device__ __forceinline__ int wrap(int a, int n) { return a - floor_div(a, n) * n; }

// ---------------------------------------------------------------------------
// population storage codec
// ---------------------------------------------------------------------------
template <int STORE>
__device__ __forceinline__ float pop_load(const Inst &P, const void *base, int q, long long idx) {
    if constexpr (STORE == 0) {
        return static_cast<const float *>(base)[q * P.n_nodes + idx];
    } else {
        const __half h = static_cast<const __half *>(base)[q * P.n_nodes + idx];
        return P.ref[q] + P.scale[q >= Q] * __half2float(h);
    }
}

// the value a population reads back as after being stored
template <int STORE>
__device__ __forceinline__ float pop_round(const Inst &P, int q, float v) {
    if constexpr (STORE == 0) {
        return v;
    } else {
        const __half h = __float2half_rn((v - P.ref[q]) * P.inv_scale[q >= Q]);
        return P.ref[q] + P.scale[q >= Q] * __half2float(h);
    }
}

template <int STORE>
__device__ __forceinline__ void pop_store(const Inst &P, void *base, int q, long long idx, float v) {
    if constexpr (STORE == 0) {
        static_cast<float *>(base)[q * P.n_nodes + idx] = v;
    } else {
        static_cast<__half *>(base)[q * P.n_nodes + idx] =
            __float2half_rn((v - P.ref[q]) * P.inv_scale[q >= Q]);
    }
}

// ---------------------------------------------------------------------------
// geometry (FP64): blending factor and rigid displacement (Sec. II.D)
// ---------------------------------------------------------------------------
// r of body k at node idx, undeformed position (X, Y): the position in the
// body's region of influence is the radial distance from its blending centre,
// or (blend_mode 1) the node's precomputed distance to the body's wall
__device__ __forceinline__ double blend_factor(const Inst &P, int k, long long idx, double X,
                                               double Y) {
    const Body &b = P.body[k];
    if (!b.present) return 1.0;
    double d;
    if (b.blend_mode == 1) {
        d = P.wall_dist[k * P.n_nodes + idx];
    } else {
        const double dx = X - b.cx, dy = Y - b.cy;
        const double d2 = dx * dx + dy * dy;
        // outside the region of influence, or in the rigid zone, without the
        // root (r_5 is flat to third order at both ends)
        if (d2 >= b.r_blend2) return 1.0;
        if (d2 <= b.r_rigid2) return 0.0;
        d = sqrt(d2);
    }
    const double s = (d - b.r_rigid) * b.inv_width;
    if (s <= 0.0) return 0.0;
    if (s >= 1.0) return 1.0;
    return s * s * s * (10.0 + s * (-15.0 + 6.0 * s));
}

// G'(X) - X = (0, h) + (R(a) - I)(X - X_EA)
__device__ __forceinline__ void rigid_disp(const Body &b, const BodySlot &s, double X, double Y,
                                           double &dx, double &dy) {
    const double rx = X - b.ex, ry = Y - b.ey;
    dx = s.cm1 * rx - s.sa * ry;
    dy = s.h + s.sa * rx + s.cm1 * ry;
}

// ---------------------------------------------------------------------------
// D2Q9 collision (Sec. II.C).  f, g in registers, overwritten with f*, g*.
// ---------------------------------------------------------------------------
struct Moments {
    float rho, ux, uy, E, T;
};

__device__ __forceinline__ Moments moments(const float f[9], const float g[9], float Cv) {
    Moments m;
    m.rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const float jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const float jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const float G = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
    const float ir = 1.0f / m.rho;
    m.ux = jx * ir;
    m.uy = jy * ir;
    m.E = 0.5f * G * ir;
    m.T = (m.E - 0.5f * (m.ux * m.ux + m.uy * m.uy)) / Cv;
    return m;
}

__device__ __forceinline__ bool state_ok(float rho, float ux, float uy, float T) {
    // also false for NaN
    return rho > 0.0f && T > 0.0f && (1.0f - T) > 0.0f && (1.0f - T - ux * ux) > 0.0f &&
           (1.0f - T - uy * uy) > 0.0f;
}

// f^eq (product form) and g^eq (with the energy correction Psi) of a
// macroscopic state (Sec. II.C).  R = T for the FP32 hot path, double for
// initialisation.
template <typename R>
__device__ __forceinline__ void equilibria(R rho, R ux, R uy, R T, R E, R feq[9], R geq[9]) {
    const R half = R(0.5), one = R(1), two = R(2);
    const R px[3] = {half * (-ux + ux * ux + T), one - (ux * ux + T), half * (ux + ux * ux + T)};
    const R py[3] = {half * (-uy + uy * uy + T), one - (uy * uy + T), half * (uy + uy * uy + T)};
    const R w[3] = {half * T, one - T, half * T};
    const R invT = one / T;
    const R inv2T2 = half * invT * invT;
    const R H = E + T;                              // enthalpy (C_v + 1) T + u^2/2
    const R qx = two * rho * ux * H, qy = two * rho * uy * H;
    const R e2 = E + two * T;
    // A = R^eq - 2 rho E T I = 2 rho [(E + 2T) u u + T^2 I]
    const R Axx = two * rho * (e2 * ux * ux + T * T);
    const R Ayy = two * rho * (e2 * uy * uy + T * T);
    const R Axy = two * rho * e2 * ux * uy;
    // Psi: delta R_a = rho (1 - 3T)(T^2 + 2 u_a^2 T + E u_a^2) / T
    const R c13 = rho * (one - R(3) * T) * invT;
    const R dRx = c13 * (T * T + (two * T + E) * ux * ux);
    const R dRy = c13 * (T * T + (two * T + E) * uy * uy);
    const R two_rho_E = two * rho * E;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int cx = CXK(k), cy = CYK(k);
        feq[k] = rho * px[cx + 1] * py[cy + 1];
        const R W = w[cx + 1] * w[cy + 1];
        const R contr = Axx * R(cx * cx) + Ayy * R(cy * cy) + two * Axy * R(cx * cy) - T * (Axx + Ayy);
        R psi = R(0);
        if (k == 0) psi = dRx + dRy;
        else if (cy == 0 && cx != 0) psi = -half * dRx;
        else if (cx == 0 && cy != 0) psi = -half * dRy;
        geq[k] = W * (two_rho_E + (qx * R(cx) + qy * R(cy)) * invT + contr * inv2T2) + psi;
    }
}

// fast reciprocal (hardware v_rcp_f32, ~1 ulp); used where a correctly
// rounded quotient is not needed
__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

// loads / stores through the global address space (the pointers live in
// device memory, so the compiler would otherwise emit flat instructions)
typedef __attribute__((address_space(1))) const float gcfloat;
typedef __attribute__((address_space(1))) const double gcdouble;
typedef __attribute__((address_space(1))) const unsigned short gcushort;
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) unsigned short gushort;

__device__ __forceinline__ float gld(const float *p) { return *(gcfloat *)p; }
__device__ __forceinline__ double2 gld(const double2 *p) {
    gcdouble *q = (gcdouble *)p;
    return make_double2(q[0], q[1]);
}

// Values every lane of a wave shares, moved into scalar registers.  Loads from
// device memory that kernels also write (the step counter, the body states,
// the work list) come back per lane; declaring them uniform lets addresses
// built from them stay scalar.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uniform(long long v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v & 0xffffffffLL));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double uniform(double v) {
    return __longlong_as_double(uniform((long long)__double_as_longlong(v)));
}
__device__ __forceinline__ BodySlot uniform(const BodySlot &a) {
    BodySlot b;
    b.h = uniform(a.h); b.a = uniform(a.a); b.hd = uniform(a.hd); b.ad = uniform(a.ad);
    b.cm1 = uniform(a.cm1); b.sa = uniform(a.sa); b.pad0 = 0.0; b.pad1 = 0.0;
    return b;
}

// Hot-path accessors through a buffer resource: one descriptor per population
// array (wave-uniform, scalar registers), the plane of population q as the
// scalar offset q * nodes * bytes and the node as a 32-bit vector offset, so
// every load / store is a single instruction with no per-lane address
// arithmetic.  The descriptor bounds the access to the array (an offset
// outside reads 0, a store outside is dropped).  Needs 18 * nodes * 4 < 2^31
// (checked at creation).
constexpr int kBufDword3 = 0x00020000;   // gfx9 descriptor word 3: 32-bit data format

struct PopBuf {
    __amdgpu_buffer_rsrc_t r;
    int plane;                            // bytes per population plane
};

template <int STORE>
__device__ __forceinline__ PopBuf pop_buf(const Inst &P, const void *base) {
    constexpr int B = STORE == 0 ? 4 : 2;
    PopBuf b;
    // base and size through readfirstlane: the descriptor is wave-uniform by
    // construction and stays in scalar registers wherever it is carried
    b.plane = uniform((int)P.n_nodes * B);
    void *const ub = reinterpret_cast<void *>(uniform(reinterpret_cast<long long>(base)));
    b.r = __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, NPOP * b.plane, kBufDword3);
    return b;
}

// byte offset of node idx inside a plane
template <int STORE>
__device__ __forceinline__ int pop_off(int idx) {
    return idx * (STORE == 0 ? 4 : 2);
}

// raw stored bits of population q (FP32 bits, or the FP16 code zero-extended)
template <int STORE>
__device__ __forceinline__ unsigned pop_ld_raw(const PopBuf &b, int q, int off) {
    if constexpr (STORE == 0) {
        return __builtin_amdgcn_raw_buffer_load_b32(b.r, off, q * b.plane, 0);
    } else {
        return __builtin_amdgcn_raw_buffer_load_b16(b.r, off, q * b.plane, 0);
    }
}

template <int STORE>
__device__ __forceinline__ float pop_decode(const Inst &P, int q, unsigned raw) {
    if constexpr (STORE == 0) {
        return __uint_as_float(raw);
    } else {
        return P.ref[q] + P.scale[q >= Q] * __half2float(__ushort_as_half((unsigned short)raw));
    }
}

// The same decoding with the scale held in a vector register (`scale`, the
// value of P.scale[q >= Q]): the fused multiply-add then takes only one
// scalar operand (the reference) and needs no copy of it per population.
template <int STORE>
__device__ __forceinline__ float pop_decode(const Inst &P, int q, unsigned raw, float scale) {
    if constexpr (STORE == 0) {
        return __uint_as_float(raw);
    } else {
        return fmaf(scale, __half2float(__ushort_as_half((unsigned short)raw)), P.ref[q]);
    }
}

// A byte offset beyond every buffer resource here (population arrays and X
// are below 2^31 bytes): loads at it return zeros without touching memory.
constexpr int kOutside = (int)0x80000000u;

// The undeformed coordinates X as a buffer resource: node idx at byte offset
// 16 idx, one 16-byte load per node.
struct XBuf {
    __amdgpu_buffer_rsrc_t r;
};

__device__ __forceinline__ XBuf x_buf(const Inst &P) {
    XBuf b;
    void *const ub = reinterpret_cast<void *>(uniform(reinterpret_cast<long long>(P.X)));
    b.r = __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, uniform((int)(P.n_nodes * 16)), kBufDword3);
    return b;
}

__device__ __forceinline__ double2 x_ld(const XBuf &b, int off) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(b.r, off, 0, 0);
    return make_double2(__hiloint2double((int)v.y, (int)v.x), __hiloint2double((int)v.w, (int)v.z));
}

// Load of a wave-uniform value through the scalar cache, for device memory
// that only earlier kernels write (the step counter, body states, coordinates)
template <class T>
__device__ __forceinline__ T sload(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}
__device__ __forceinline__ double2 sload(const double2 *p) {
    const double *q = reinterpret_cast<const double *>(p);
    return make_double2(sload(q), sload(q + 1));
}

// Store of a new population.  NT: non-temporal (cache policy bit 1), for a
// step that streams more than the Infinity Cache holds: the new populations
// are then read again only from HBM, and keeping them out of the caches leaves
// L2 to the halo rows that later tiles of the same XCD read.  (Smaller working
// sets stay in the Infinity Cache from one step to the next, which
// non-temporal stores would forgo.)
template <int STORE, bool NT = false>
__device__ __forceinline__ void pop_st(const Inst &P, const PopBuf &b, int q, int off, float v) {
    constexpr int aux = NT ? 2 : 0;
    if constexpr (STORE == 0) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), b.r, off, q * b.plane, aux);
    } else {
        const unsigned short h =
            __half_as_ushort(__float2half_rn((v - P.ref[q]) * P.inv_scale[q >= Q]));
        __builtin_amdgcn_raw_buffer_store_b16(h, b.r, off, q * b.plane, aux);
    }
}

// Collision at one node (Sec. II.C, kinetic equations):
//   f* = f + omega (f^eq - f) + dt phi,  phi_i = -(W_i/T) c_i . F
//   g* = g + omega (g^eq - g) + (omega_1 - omega)(g^* - g)
//      = g + omega_1 (g^eq - g) + (omega_1 - omega) W_i (q^* - q^eq) . c_i / T
// with q^* - q^eq = 2 u . (P - P^eq).
__device__ __forceinline__ void collide(float f[9], float g[9], float Fx, float Fy, const Inst &P,
                                        unsigned &err) {
    // moments from sums and differences of opposite populations
    const float s13 = f[1] + f[3], d13 = f[1] - f[3];
    const float s24 = f[2] + f[4], d24 = f[2] - f[4];
    const float s56 = f[5] + f[6], d56 = f[5] - f[6];
    const float s78 = f[7] + f[8], d78 = f[7] - f[8];
    const float sd = s56 + s78;                        // the four diagonal populations
    const float rho = (f[0] + s13) + (s24 + sd);
    const float jx = d13 + (d56 - d78);
    const float jy = d24 + (s56 - s78);
    const float Pxx = s13 + sd, Pyy = s24 + sd, Pxy = d56 + d78;
    const float G = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
    const float ir = rcpf(rho);
    const float ux = jx * ir, uy = jy * ir;
    const float uxx = ux * ux, uyy = uy * uy;
    const float E = 0.5f * G * ir;
    const float T = (E - 0.5f * (uxx + uyy)) * (P.gamma - 1.0f);
    if (!state_ok(rho, ux, uy, T)) err |= ERR_STATE;
    // omega from mu = (1/omega - 1/2) p dt; Pr = (1/omega - 1/2)/(1/omega_1 - 1/2)
    const float a = P.mu * rcpf(rho * T * P.dt);
    const float omega = rcpf(a + 0.5f);
    const float omega1 = rcpf(a * rcpf(P.Pr) + 0.5f);
    const float invT = rcpf(T);
    // lattice weights: axis (1 - T) T/2, diagonal (T/2)^2 (the rest population's
    // equilibria follow from the closure below)
    const float wh = 0.5f * T, w1 = 1.0f - T;
    const float Wa = w1 * wh, Wd = wh * wh;
    // product-form f^eq = rho px[cx] py[cy], px[+-1] = (u^2 + T +- u)/2, px[0] = 1 - u^2 - T
    const float hx = 0.5f * (uxx + T), hy = 0.5f * (uyy + T);
    const float rpm = rho * (hx - 0.5f * ux), rpp = rho * (hx + 0.5f * ux), rp0 = rho * (1.0f - 2.0f * hx);
    const float pym = hy - 0.5f * uy, pyp = hy + 0.5f * uy, py0 = 1.0f - 2.0f * hy;
    float feq[9];
    feq[0] = rp0 * py0;
    feq[1] = rpp * py0;
    feq[2] = rp0 * pyp;
    feq[3] = rpm * py0;
    feq[4] = rp0 * pym;
    feq[5] = rpp * pyp;
    feq[6] = rpm * pyp;
    feq[7] = rpm * pym;
    feq[8] = rpp * pym;
    // g^eq (with Psi): W_i [2 rho E + q^eq.c_i/T + A:(c_i c_i - T I)/(2T^2)] + Psi_i,
    // q^eq = 2 rho u H, H = E + T; A = 2 rho [(E + 2T) u u + T^2 I]
    const float inv2T2 = 0.5f * invT * invT;
    const float H = E + T;
    const float qxT = 2.0f * rho * ux * H * invT, qyT = 2.0f * rho * uy * H * invT;
    const float e2 = E + 2.0f * T;
    const float Axx = 2.0f * rho * (e2 * uxx + T * T);
    const float Ayy = 2.0f * rho * (e2 * uyy + T * T);
    const float Axy = 2.0f * rho * e2 * ux * uy;
    // Psi: delta R_a = rho (1 - 3T)(T^2 + 2 u_a^2 T + E u_a^2) / T
    const float c13 = rho * (1.0f - 3.0f * T) * invT;
    const float dRx = c13 * (T * T + (2.0f * T + E) * uxx);
    const float dRy = c13 * (T * T + (2.0f * T + E) * uyy);
    const float two_rho_E = 2.0f * rho * E;
    const float trA = T * (Axx + Ayy);
    const float w[3] = {wh, w1, wh};
    float geq[9];
#pragma unroll
    for (int k = 1; k < 9; ++k) {
        const int cx = CXK(k), cy = CYK(k);
        const float W = w[cx + 1] * w[cy + 1];
        const float contr = Axx * (float)(cx * cx) + Ayy * (float)(cy * cy) +
                            2.0f * Axy * (float)(cx * cy) - trA;
        float psi = 0.0f;
        if (cy == 0) psi = -0.5f * dRx;
        else if (cx == 0) psi = -0.5f * dRy;
        geq[k] = W * (two_rho_E + qxT * (float)cx + qyT * (float)cy + contr * inv2T2) + psi;
    }
    // Close the conserved moments of the equilibria on the stored moments, so
    // FP32 rounding of the product form cannot make mass, momentum or energy
    // drift coherently over many steps (the same identities, evaluated so that
    // sum f^eq = rho, sum f^eq c = rho u and sum g^eq = 2 rho E hold to one rounding).
    feq[1] = jx + ((feq[3] + feq[6] + feq[7]) - (feq[5] + feq[8]));
    feq[2] = jy + ((feq[4] + feq[7] + feq[8]) - (feq[5] + feq[6]));
    feq[0] = rho - (((feq[1] + feq[2]) + (feq[3] + feq[4])) + ((feq[5] + feq[6]) + (feq[7] + feq[8])));
    geq[0] = G - (((geq[1] + geq[2]) + (geq[3] + geq[4])) + ((geq[5] + geq[6]) + (geq[7] + geq[8])));
    // Collision (Sec. II.C, kinetic equations), the forcing terms by direction:
    //   f* = f + omega (f^eq - f) + dt phi,  phi_i = -(W_i/T) c_i . F
    //   g* = g + omega_1 (g^eq - g) + (omega_1 - omega) W_i (q^* - q^eq) . c_i / T,
    //   q^* - q^eq = 2 u . (P - P^eq)
    const float dPxx = Pxx - rho * (T + uxx);
    const float dPyy = Pyy - rho * (T + uyy);
    const float dPxy = Pxy - rho * ux * uy;
    const float cf = -P.dt * invT, cgm = 2.0f * (omega1 - omega) * invT;
    const float vfx = cf * Fx, vfy = cf * Fy;
    const float vgx = cgm * (ux * dPxx + uy * dPxy), vgy = cgm * (ux * dPxy + uy * dPyy);
    const float tfx = Wa * vfx, tfy = Wa * vfy, tfp = Wd * (vfx + vfy), tfm = Wd * (vfx - vfy);
    const float tgx = Wa * vgx, tgy = Wa * vgy, tgp = Wd * (vgx + vgy), tgm = Wd * (vgx - vgy);
    const float tf[9] = {0.0f, tfx, tfy, -tfx, -tfy, tfp, -tfm, -tfp, tfm};
    const float tg[9] = {0.0f, tgx, tgy, -tgx, -tgy, tgp, -tgm, -tgp, tgm};
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        f[k] = f[k] + omega * (feq[k] - f[k]) + tf[k];
        g[k] = g[k] + omega1 * (geq[k] - g[k]) + tg[k];
    }
}

// launch a kernel template for the storage format (0 FP32, 1 FP16 shifted)
#define FSI_DISPATCH(storage, KERNEL, GRID, BLOCK, STREAM, ...)                              \
    do {                                                                                 \
        if ((storage) == 0) hipLaunchKernelGGL(KERNEL<0>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); \
        else hipLaunchKernelGGL(KERNEL<1>, GRID, BLOCK, 0, STREAM, __VA_ARGS__);          \
    } while (0)

}  // namespace fsi
