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
        d = sqrt(dx * dx + dy * dy);
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
    b.plane = (int)P.n_nodes * B;
    b.r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, NPOP * b.plane,
                                            kBufDword3);
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

template <int STORE>
__device__ __forceinline__ void pop_st(const Inst &P, const PopBuf &b, int q, int off, float v) {
    if constexpr (STORE == 0) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), b.r, off, q * b.plane, 0);
    } else {
        const unsigned short h =
            __half_as_ushort(__float2half_rn((v - P.ref[q]) * P.inv_scale[q >= Q]));
        __builtin_amdgcn_raw_buffer_store_b16(h, b.r, off, q * b.plane, 0);
    }
}

// Collision at one node (Sec. II.C, kinetic equations):
//   f* = f + omega (f^eq - f) + dt phi,  phi_i = -(W_i/T) c_i . F
//   g* = g + omega (g^eq - g) + (omega_1 - omega)(g^* - g)
//      = g + omega_1 (g^eq - g) + (omega_1 - omega) W_i (q^* - q^eq) . c_i / T
// with q^* - q^eq = 2 u . (P - P^eq).
__device__ __forceinline__ void collide(float f[9], float g[9], float Fx, float Fy, const Inst &P,
                                        unsigned &err) {
    const float rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const float jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const float jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const float G = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
    const float ir = rcpf(rho);
    const float ux = jx * ir, uy = jy * ir;
    const float E = 0.5f * G * ir;
    const float T = (E - 0.5f * (ux * ux + uy * uy)) * (P.gamma - 1.0f);
    if (!state_ok(rho, ux, uy, T)) err |= ERR_STATE;
    const float Pxx = (f[1] + f[3]) + (f[5] + f[6]) + (f[7] + f[8]);
    const float Pyy = (f[2] + f[4]) + (f[5] + f[6]) + (f[7] + f[8]);
    const float Pxy = (f[5] - f[6]) + (f[7] - f[8]);
    // omega from mu = (1/omega - 1/2) p dt; Pr = (1/omega - 1/2)/(1/omega_1 - 1/2)
    const float a = P.mu * rcpf(rho * T * P.dt);
    const float omega = rcpf(a + 0.5f);
    const float omega1 = rcpf(a * rcpf(P.Pr) + 0.5f);
    const float invT = rcpf(T);
    // equilibria (product-form f^eq; g^eq with Psi)
    const float px[3] = {0.5f * (-ux + ux * ux + T), 1.0f - (ux * ux + T), 0.5f * (ux + ux * ux + T)};
    const float py[3] = {0.5f * (-uy + uy * uy + T), 1.0f - (uy * uy + T), 0.5f * (uy + uy * uy + T)};
    const float w[3] = {0.5f * T, 1.0f - T, 0.5f * T};
    const float inv2T2 = 0.5f * invT * invT;
    const float H = E + T;
    const float qx = 2.0f * rho * ux * H, qy = 2.0f * rho * uy * H;
    const float e2 = E + 2.0f * T;
    const float Axx = 2.0f * rho * (e2 * ux * ux + T * T);
    const float Ayy = 2.0f * rho * (e2 * uy * uy + T * T);
    const float Axy = 2.0f * rho * e2 * ux * uy;
    const float c13 = rho * (1.0f - 3.0f * T) * invT;
    const float dRx = c13 * (T * T + (2.0f * T + E) * ux * ux);
    const float dRy = c13 * (T * T + (2.0f * T + E) * uy * uy);
    const float two_rho_E = 2.0f * rho * E;
    const float trA = T * (Axx + Ayy);
    const float dPxx = Pxx - rho * (T + ux * ux);
    const float dPyy = Pyy - rho * (T + uy * uy);
    const float dPxy = Pxy - rho * ux * uy;
    const float dqx = 2.0f * (ux * dPxx + uy * dPxy);
    const float dqy = 2.0f * (ux * dPxy + uy * dPyy);
    // per-direction vectors: f gets -dt F/T, g gets (omega_1 - omega) dq/T + q^eq/T
    const float cf = -P.dt * invT, cg = (omega1 - omega) * invT;
    const float vfx = cf * Fx, vfy = cf * Fy;
    const float vgx = cg * dqx, vgy = cg * dqy;
    const float qxT = qx * invT, qyT = qy * invT;
    float feq[9], geq[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int cx = CXK(k), cy = CYK(k);
        const float W = w[cx + 1] * w[cy + 1];
        feq[k] = rho * px[cx + 1] * py[cy + 1];
        const float contr = Axx * (float)(cx * cx) + Ayy * (float)(cy * cy) +
                            2.0f * Axy * (float)(cx * cy) - trA;
        float psi = 0.0f;
        if (k == 0) psi = dRx + dRy;
        else if (cy == 0) psi = -0.5f * dRx;
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
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int cx = CXK(k), cy = CYK(k);
        const float W = w[cx + 1] * w[cy + 1];
        f[k] = f[k] + omega * (feq[k] - f[k]) + W * (vfx * (float)cx + vfy * (float)cy);
        g[k] = g[k] + omega1 * (geq[k] - g[k]) + W * (vgx * (float)cx + vgy * (float)cy);
    }
}

// launch a kernel template for the storage format (0 FP32, 1 FP16 shifted)
#define FSI_DISPATCH(storage, KERNEL, GRID, BLOCK, STREAM, ...)                              \
    do {                                                                                 \
        if ((storage) == 0) hipLaunchKernelGGL(KERNEL<0>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); \
        else hipLaunchKernelGGL(KERNEL<1>, GRID, BLOCK, 0, STREAM, __VA_ARGS__);          \
    } while (0)

}  // namespace fsi
