// Per-cell arithmetic of the cascaded central-moment LBM on D2Q9, the
// lattice the paper derives (Secs. 2-11), in the same factorised
// central-moment form as the D3Q27 code: two axis passes of the 3-point
// transform, the source recursion of the exact identity, relaxation towards
// kappa^M - sigma/2 with the paper's rates omega_3 (trace), omega_4 = omega_5
// (shear), omega_6 (xxy), omega_7 (xyy), omega_8 (xxyy), exact inverse.
//
// Internal indices: population i = (ex+1) + 3 (ey+1); moment p = a + 3 b.
// Deviation ("well-conditioned") variables as in cm_math.hpp.
#pragma once
#include "cm_math.hpp"

namespace cm2 {
using cm::fwd3;
using cm::inv3;
using cm::r1;
using cm::w1;
#if !defined(__HIPCC__)
using std::sqrt;
#endif

template <typename R> CM_HD constexpr R w9(int i) { return w1<R>(i % 3) * w1<R>(i / 3); }
template <typename R> CM_HD constexpr R unit9(int p) { return r1<R>(p % 3) * r1<R>(p / 3); }
CM_HD constexpr int J(int a, int b) { return a + 3 * b; }

// The paper's velocity index alpha (Sec. 2: rest, (1,0), (0,1), (-1,0),
// (0,-1), (1,1), (-1,1), (-1,-1), (1,-1)) -> internal index (ex+1) + 3 (ey+1).
CM_HD constexpr int from_paper(int a) {
    return a == 0 ? 4 : a == 1 ? 5 : a == 2 ? 7 : a == 3 ? 3 : a == 4 ? 1 : a == 5 ? 8 : a == 6 ? 6 : a == 7 ? 0 : 2;
}

// Rates in the paper's D2Q9 numbering.
template <typename R>
struct Rates2 {
    R rho0;
    R w3;        // trace of the second-order moments (bulk)
    R ws;        // omega_4 = omega_5 (shear)
    R w6, w7, w8;
    R tau0, smag;
    int rc, fact;
    R sgs;       // sub-grid stress as a force (Sec. 14): C_s^2 omega0^2 / (2 cs^4)
};

template <typename R>
CM_HD void forward9(R (&m)[9], R ux, R uy, R rho0) {
#pragma unroll
    for (int ix = 0; ix < 3; ++ix) fwd3(m[ix], m[ix + 3], m[ix + 6], uy, rho0, w1<R>(ix));
#pragma unroll
    for (int cy = 0; cy < 3; ++cy) fwd3(m[3 * cy], m[3 * cy + 1], m[3 * cy + 2], ux, rho0, r1<R>(cy));
}

template <typename R>
CM_HD void inverse9(R (&m)[9], R ux, R uy, R rho0) {
#pragma unroll
    for (int cy = 0; cy < 3; ++cy) inv3(m[3 * cy], m[3 * cy + 1], m[3 * cy + 2], ux, rho0, r1<R>(cy));
#pragma unroll
    for (int ix = 0; ix < 3; ++ix) inv3(m[ix], m[ix + 3], m[ix + 6], uy, rho0, w1<R>(ix));
}

// h: deviation populations in, post-collision deviations out.
// SGS (Sec. 14 coupling): the force is F + rho acc (acc = -div R of the
// previous step) and this step's sub-grid stress is returned in st
// (xx, yy, xy): R^d = sgs Q Pi^d / rho^2, Q = sqrt(2 Pi^d : Pi^d).
template <typename R, bool LES, bool VAR = false, bool SGS = false>
CM_HD void collide9(R (&h)[9], R Fx, R Fy, const Rates2<R>& P, R& rho_out, R& ux_out, R& uy_out,
                    const R* acc = nullptr, R* st = nullptr) {
    R drho = R(0), jx = R(0), jy = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        drho += h[i];
        jx += R(i % 3 - 1) * h[i];
        jy += R(i / 3 - 1) * h[i];
    }
    const R rho = P.rho0 + drho;
    const R inv_rho = R(1) / rho;
    R inv_rho_u = inv_rho;
    if constexpr (VAR) inv_rho_u = P.rc ? R(1) / P.rho0 : inv_rho;
    if constexpr (SGS) {
        Fx += rho * acc[0];
        Fy += rho * acc[1];
    }
    const R ux = (jx + R(0.5) * Fx) * inv_rho_u;
    const R uy = (jy + R(0.5) * Fy) * inv_rho_u;
    forward9(h, ux, uy, P.rho0);
    // sources (first-order kappa of f are zero, so second-order sigma vanish)
    const R fx = Fx * inv_rho, fy = Fy * inv_rho;
    const R third = R(1) / R(3), ninth = R(1) / R(9), half = R(0.5);
    const R k20 = h[J(2, 0)] + P.rho0 * third, k02 = h[J(0, 2)] + P.rho0 * third, k11 = h[J(1, 1)];
    const R s21 = R(2) * fx * k11 + fy * k20;
    const R s12 = fx * k02 + R(2) * fy * k11;
    const R k21 = h[J(2, 1)] + half * s21, k12 = h[J(1, 2)] + half * s12;
    const R s22 = R(2) * (fx * k12 + fy * k21);
    if constexpr (SGS) {
        const R dxx = half * (h[J(2, 0)] - h[J(0, 2)]), xy = h[J(1, 1)];
        const R c = P.sgs * sqrt(R(2) * (R(2) * dxx * dxx + R(2) * xy * xy)) * inv_rho_u * inv_rho_u;
        st[0] = c * dxx;
        st[1] = -(c * dxx);
        st[2] = c * xy;
    }
    R ws = P.ws;
    if constexpr (LES) {
        const R dxx = half * (h[J(2, 0)] - h[J(0, 2)]);   // traceless part (2D): +-(xx - yy)/2
        const R q = sqrt(R(2) * (R(2) * dxx * dxx + R(2) * k11 * k11));
        const R tau = half * (P.tau0 + sqrt(P.tau0 * P.tau0 + P.smag * q * inv_rho_u));
        ws = R(1) / tau;
    }
    // second order: trace with omega_3, xx - yy and xy with the shear rate
    const R dx = drho * third - h[J(2, 0)], dy = drho * third - h[J(0, 2)];
    const R tr = half * (P.w3 + ws), df = half * (P.w3 - ws);
    const R qx = h[J(2, 0)] + tr * dx + df * dy;   // post-collision deviations of xx and yy
    const R qy = h[J(0, 2)] + df * dx + tr * dy;
    h[J(2, 0)] = qx;
    h[J(0, 2)] = qy;
    h[J(1, 1)] -= ws * h[J(1, 1)];
    // third order
    h[J(2, 1)] += P.w6 * (-half * s21 - h[J(2, 1)]) + s21;
    h[J(1, 2)] += P.w7 * (-half * s12 - h[J(1, 2)]) + s12;
    // fourth order: Maxwellian drho/9, or the factorized product (Sec. 13)
    R a22 = drho * ninth;
    if constexpr (VAR) {
        if (P.fact) a22 = (-P.rho0 * drho * ninth + P.rho0 * third * (qx + qy) + qx * qy) * inv_rho;
    }
    h[J(2, 2)] += P.w8 * (a22 - half * s22 - h[J(2, 2)]) + s22;
    // first order: kappabar_1 + F (= +F/2 unless reduced compressibility)
    bool rc = false;
    if constexpr (VAR) rc = P.rc != 0;
    if (rc) {
        h[J(1, 0)] += Fx;
        h[J(0, 1)] += Fy;
    } else {
        h[J(1, 0)] = half * Fx;
        h[J(0, 1)] = half * Fy;
    }
    inverse9(h, ux, uy, P.rho0);
    rho_out = rho;
    ux_out = ux;
    uy_out = uy;
}

template <typename R>
CM_HD void equilibrium9(R (&h)[9], R rho, R ux, R uy, R Fx, R Fy, R rho0, bool rc) {
    const R drho = rho - rho0;
#pragma unroll
    for (int p = 0; p < 9; ++p) h[p] = drho * unit9<R>(p);
    // sigma(kappa^M): only moments with one exponent equal to 1
    h[J(1, 0)] -= R(0.5) * Fx;
    h[J(0, 1)] -= R(0.5) * Fy;
    h[J(1, 2)] -= R(0.5) * Fx * r1<R>(2);
    h[J(2, 1)] -= R(0.5) * Fy * r1<R>(2);
    if (rc) {
        h[J(1, 0)] -= drho * ux;
        h[J(0, 1)] -= drho * uy;
    }
    inverse9(h, ux, uy, rho0);
}

}  // namespace cm2
