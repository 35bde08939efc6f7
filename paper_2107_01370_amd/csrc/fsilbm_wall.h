// Wall-node arithmetic shared by the structured and the unstructured wall
// kernels: Grad's populations for the missing populations (Sec. III.A.1) and
// the FP64 stress of a complete wall node (Sec. III force).  Included by the
// kernel sources only.
#pragma once

#include "fsilbm_device.h"

namespace fsi {

// Grad's approximation f_k = f_k^eq + dt f_k^(1), g_k = g_k^eq + dt g_k^(1) of
// the populations flagged in `miss`, from the targets (rho_t, u_t, T_t, E_t)
// and the gradients d_a of u_x, u_y, T, E at the wall node; the others are
// left as they are.
__device__ __forceinline__ void grad_populations(const Inst &P, unsigned miss, float rho_t, float ux_t,
                                                 float uy_t, float T_t, float E_t, float duxx,
                                                 float duxy, float duyx, float duyy, float dTx,
                                                 float dTy, float dEx, float dEy, float f[9],
                                                 float g[9]) {
    const float Cv = P.Cv, Cp = P.Cp, dt = P.dt;
    const float aa = P.mu / (rho_t * T_t * dt);
    const float omega = 1.0f / (aa + 0.5f);
    const float omega1 = 1.0f / (aa / P.Pr + 0.5f);
    // S = grad u + grad u^T, (grad u)_ab = d_a u_b
    const float Sxx = 2.0f * duxx, Syy = 2.0f * duyy, Sxy = duxy + duyx;
    const float div = duxx + duyy;
    const float pref = -rho_t * T_t / omega;
    const float P1xx = pref * (Sxx - div / Cv);
    const float P1yy = pref * (Syy - div / Cv);
    const float P1xy = pref * Sxy;
    const float q1x = -(2.0f / omega1) * rho_t * Cp * T_t * dTx + 2.0f * (ux_t * P1xx + uy_t * P1xy);
    const float q1y = -(2.0f / omega1) * rho_t * Cp * T_t * dTy + 2.0f * (ux_t * P1xy + uy_t * P1yy);
    const float rpref = -(2.0f / omega1) * rho_t * T_t;
    const float e2 = E_t + 2.0f * T_t;
    const float R1xx = rpref * (Sxx * e2 + 2.0f * ux_t * dEx);
    const float R1yy = rpref * (Syy * e2 + 2.0f * uy_t * dEy);
    const float R1xy = rpref * (Sxy * e2 + ux_t * dEy + uy_t * dEx);
    float feq[9], geq[9];
    equilibria<float>(rho_t, ux_t, uy_t, T_t, E_t, feq, geq);
    const float w[3] = {0.5f * T_t, 1.0f - T_t, 0.5f * T_t};
    const float invT = 1.0f / T_t, inv2T2 = 0.5f * invT * invT;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if (!(miss & (1u << k))) continue;
        const int cx = CXK(k), cy = CYK(k);
        const float W = w[cx + 1] * w[cy + 1];
        const float ccx = (float)(cx * cx) - T_t, ccy = (float)(cy * cy) - T_t;
        const float cxy = 2.0f * (float)(cx * cy);
        const float fneq = W * (P1xx * ccx + P1yy * ccy + P1xy * cxy) * inv2T2;
        const float gneq = W * ((q1x * (float)cx + q1y * (float)cy) * invT +
                                (R1xx * ccx + R1yy * ccy + R1xy * cxy) * inv2T2);
        f[k] = feq[k] + dt * fneq;
        g[k] = geq[k] + dt * gneq;
    }
}

// sigma = -p I - (1 - omega/2) sum (f - f^eq) c c of a complete wall node, with
// the moments formed in FP64 from its populations; returns (s_xx, s_xy, s_yy)
// and whether the state is physical
__device__ __forceinline__ bool wall_stress(const Inst &P, const float f[9], const float g[9],
                                            double &sxx, double &sxy, double &syy) {
    const float Cv = P.Cv;
    double fd[9], gd[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        fd[k] = f[k];
        gd[k] = g[k];
    }
    double rho = 0, jx = 0, jy = 0, G = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        rho += fd[k];
        jx += CXK(k) * fd[k];
        jy += CYK(k) * fd[k];
        G += gd[k];
    }
    const double ux = jx / rho, uy = jy / rho, E = 0.5 * G / rho;
    const double T = (E - 0.5 * (ux * ux + uy * uy)) / (double)Cv;
    double feq[9], geq[9];
    equilibria<double>(rho, ux, uy, T, E, feq, geq);
    double Pxx = 0.0, Pyy = 0.0, Pxy = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double d = fd[k] - feq[k];
        const int cx = CXK(k), cy = CYK(k);
        Pxx += d * (double)(cx * cx);
        Pyy += d * (double)(cy * cy);
        Pxy += d * (double)(cx * cy);
    }
    const double p = rho * T;
    const double omega = 1.0 / ((double)P.mu / (p * P.dt_d) + 0.5);
    const double kk = 1.0 - 0.5 * omega;
    sxx = -p - kk * Pxx;
    syy = -p - kk * Pyy;
    sxy = -kk * Pxy;
    return state_ok((float)rho, (float)ux, (float)uy, (float)T);
}

}  // namespace fsi
