// Per-cell arithmetic of the cascaded central-moment LBM on D3Q27.
//
// Conventions
//   population index  i = (ex+1) + 3 (ey+1) + 9 (ez+1)
//   moment index      p = a + 3 b + 9 c   for exponents (a, b, c) in {0,1,2}^3
// The 27 central moments about the local velocity are obtained by three
// one-dimensional three-point transforms (z, then y, then x lines). This is the
// binomial frame change of the paper (Eq. binomialtheorem) factorised by axis,
// which the tensor-product lattice allows.
//
// All quantities are carried as deviations from the rest state rho0 * w_i
// ("well-conditioned" form): a line transform takes the rest-state mass K of
// its line, so that the outputs are central moments minus rho0 times the unit
// Maxwellian moments r(a) r(b) r(c), r = (1, 0, 1/3). This keeps the small
// non-equilibrium parts of the state from being swamped by the O(1) rest
// state in single or half precision.
//
// The same header compiles for the host (without HIP) so that the arithmetic
// can be checked on the CPU.
#pragma once
#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define CM_HD __host__ __device__ __forceinline__
#else
#include <cmath>
#define CM_HD inline
#endif

namespace cm {
#if !defined(__HIPCC__)
using std::sqrt;
#endif

// 1D rest weights for e = -1, 0, +1 and unit Maxwellian moments of order 0, 1, 2
// Fused multiply-add a * b + c with one rounding.
template <typename R> CM_HD R fmad(R a, R b, R c) {
#if defined(__HIPCC__)
    return fma(a, b, c);
#else
    return std::fma(a, b, c);
#endif
}

// Reciprocal and square root. With FAST in single precision on the GPU they
// are the hardware instructions (within 1 ulp) rather than the correctly
// rounded sequences (about ten instructions each); the FP16-storage kernels,
// which are bound by instruction issue, use them. On the host, and for double
// precision, they are exact.
template <bool FAST, typename R> CM_HD R rcp_(R x) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (FAST && sizeof(R) == 4) return __builtin_amdgcn_rcpf(x);
#endif
    return R(1) / x;
}
template <bool FAST, typename R> CM_HD R sqrt_(R x) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (FAST && sizeof(R) == 4) return __builtin_amdgcn_sqrtf(x);
#endif
    return sqrt(x);
}

template <typename R> CM_HD constexpr R w1(int s) { return s == 1 ? R(2) / R(3) : R(1) / R(6); }
template <typename R> CM_HD constexpr R r1(int k) { return k == 0 ? R(1) : (k == 1 ? R(0) : R(1) / R(3)); }
template <typename R> CM_HD constexpr R w27(int i) { return w1<R>(i % 3) * w1<R>((i / 3) % 3) * w1<R>(i / 9); }
template <typename R> CM_HD constexpr R unit27(int p) { return r1<R>(p % 3) * r1<R>((p / 3) % 3) * r1<R>(p / 9); }
// v + rho0 r(a)r(b)r(c) for moment p, leaving the term out where it is zero
// (any odd exponent): the compiler may not drop an added rho0 * 0 itself.
template <typename R> CM_HD R plus_rest(R v, R rho0, int p) { return unit27<R>(p) != R(0) ? v + rho0 * unit27<R>(p) : v; }

CM_HD constexpr int I(int a, int b, int c) { return a + 3 * b + 9 * c; }
CM_HD constexpr int ord(int p) { return p % 3 + (p / 3) % 3 + p / 9; }
CM_HD constexpr int ex_(int p, int d) { return d == 0 ? p % 3 : (d == 1 ? (p / 3) % 3 : p / 9); }
CM_HD constexpr int lower(int p, int d) { return d == 0 ? p - 1 : (d == 1 ? p - 3 : p - 9); }

// Moments of total order >= 3, in ascending order (the source recursion order).
CM_HD constexpr int high(int k) {
    switch (k) {
        case 0: return I(2, 1, 0);
        case 1: return I(2, 0, 1);
        case 2: return I(1, 2, 0);
        case 3: return I(0, 2, 1);
        case 4: return I(1, 0, 2);
        case 5: return I(0, 1, 2);
        case 6: return I(1, 1, 1);
        case 7: return I(2, 2, 0);
        case 8: return I(2, 0, 2);
        case 9: return I(0, 2, 2);
        case 10: return I(2, 1, 1);
        case 11: return I(1, 2, 1);
        case 12: return I(1, 1, 2);
        case 13: return I(2, 2, 1);
        case 14: return I(2, 1, 2);
        case 15: return I(1, 2, 2);
        default: return I(2, 2, 2);
    }
}

// ------------------------------------------------------------ line transforms
// Forward: values at e = -1, 0, +1 (deviations from K * w1) -> central moments
// of order 0, 1, 2 about u (deviations from K * r1).
template <typename R>
CM_HD void fwd3(R& a, R& b, R& c, R u, R rho0, R cK) {
    const R s = a + c;
    const R d = c - a;
    const R k0 = s + b;
    const R kf = cK == R(0) ? k0 : k0 + rho0 * cK;   // rest mass K = rho0 cK, cK a constant
    const R k1 = d - u * kf;
    const R k2 = s - u * (d + k1);   // s - 2 u d + u^2 kf
    a = k0; b = k1; c = k2;
}

// Inverse of fwd3 for the same u and K.
template <typename R>
CM_HD void inv3(R& a, R& b, R& c, R u, R rho0, R cK) {
    const R k0 = a, k1 = b, k2 = c;
    const R kf = cK == R(0) ? k0 : k0 + rho0 * cK;
    const R m1 = k1 + u * kf;
    const R m2 = k2 + u * (k1 + m1);   // k2 + 2 u k1 + u^2 kf
    const R hp = R(0.5) * (m2 + m1);
    a = hp - m1;
    b = k0 - m2;
    c = hp;
}

// Transpose of the linear part of fwd3: moment-space adjoints (mu0, mu1, mu2)
// -> value-space adjoints v_e = mu0 + (e-u) mu1 + (e-u)^2 mu2.
template <typename R>
CM_HD void fwd3_T(R& a, R& b, R& c, R u) {
    const R m0 = a, m1 = b, m2 = c;
    const R em = R(-1) - u, e0 = -u, ep = R(1) - u;
    a = m0 + em * (m1 + em * m2);
    b = m0 + e0 * (m1 + e0 * m2);
    c = m0 + ep * (m1 + ep * m2);
}

// Transpose of the linear part of inv3: value-space adjoints (l-, l0, l+)
// -> moment-space adjoints.
template <typename R>
CM_HD void inv3_T(R& a, R& b, R& c, R u) {
    const R lm = a, l0 = b, lp = c;
    const R mu2 = R(0.5) * (lp + lm) - l0;
    const R mu1 = R(0.5) * (lp - lm) + R(2) * u * mu2;
    const R mu0 = l0 + u * (mu1 - u * mu2);
    a = mu0; b = mu1; c = mu2;
}

template <typename R>
CM_HD void forward_transform(R (&m)[27], R ux, R uy, R uz, R rho0) {
#pragma unroll
    for (int iy = 0; iy < 3; ++iy)
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) {
            const int b = ix + 3 * iy;
            fwd3(m[b], m[b + 9], m[b + 18], uz, rho0, w1<R>(ix) * w1<R>(iy));
        }
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) {
            const int b = ix + 9 * cz;
            fwd3(m[b], m[b + 3], m[b + 6], uy, rho0, w1<R>(ix) * r1<R>(cz));
        }
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int cy = 0; cy < 3; ++cy) {
            const int b = 3 * cy + 9 * cz;
            fwd3(m[b], m[b + 1], m[b + 2], ux, rho0, r1<R>(cy) * r1<R>(cz));
        }
}

template <typename R>
CM_HD void inverse_transform(R (&m)[27], R ux, R uy, R uz, R rho0) {
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int cy = 0; cy < 3; ++cy) {
            const int b = 3 * cy + 9 * cz;
            inv3(m[b], m[b + 1], m[b + 2], ux, rho0, r1<R>(cy) * r1<R>(cz));
        }
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) {
            const int b = ix + 9 * cz;
            inv3(m[b], m[b + 3], m[b + 6], uy, rho0, w1<R>(ix) * r1<R>(cz));
        }
#pragma unroll
    for (int iy = 0; iy < 3; ++iy)
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) {
            const int b = ix + 3 * iy;
            inv3(m[b], m[b + 9], m[b + 18], uz, rho0, w1<R>(ix) * w1<R>(iy));
        }
}

// The per-axis matrices act on different axes and commute, so the transposes
// can be applied axis by axis in any order.
template <typename R>
CM_HD void forward_transform_T(R (&v)[27], R ux, R uy, R uz) {
#pragma unroll
    for (int k = 0; k < 9; ++k) fwd3_T(v[3 * k], v[3 * k + 1], v[3 * k + 2], ux);
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) fwd3_T(v[ix + 9 * cz], v[ix + 9 * cz + 3], v[ix + 9 * cz + 6], uy);
#pragma unroll
    for (int k = 0; k < 9; ++k) fwd3_T(v[k], v[k + 9], v[k + 18], uz);
}

template <typename R>
CM_HD void inverse_transform_T(R (&v)[27], R ux, R uy, R uz) {
#pragma unroll
    for (int k = 0; k < 9; ++k) inv3_T(v[k], v[k + 9], v[k + 18], uz);
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) inv3_T(v[ix + 9 * cz], v[ix + 9 * cz + 3], v[ix + 9 * cz + 6], uy);
#pragma unroll
    for (int k = 0; k < 9; ++k) inv3_T(v[3 * k], v[3 * k + 1], v[3 * k + 2], ux);
}

// ------------------------------------------------------------ rates
template <typename R>
struct Rates {
    R rho0;
    R ws, wb;            // shear and bulk rates (second order)
    R w3a, w3b, w3c;     // third order: (xyy+xzz)-type, (xyy-xzz)-type, xyz
    R w4a, w4b;          // fourth order: xxyy-type, xxyz-type
    R w5, w6;
    R tau0;              // 1 / ws
    R smag;              // 2 Cs^2 / cs^4 = 18 Cs^2 (0 disables the eddy viscosity)
    int rc;              // reduced compressibility (Sec. 12): rho0 u = sum fbar e + F/2
    int fact;            // factorized fourth/sixth-order attractors (Sec. 13)
    R sgs;               // sub-grid stress as a force (Sec. 14): C_s^2 omega0^2 / (2 cs^4)
    // Coefficients of the closed-form relaxation of the orders >= 3 (set by
    // derive_coefficients from the rates above): a moment relaxed with rate w
    // becomes (1 - w) m + w a + (1 - w/2) sigma (a its attractor), written
    // scaled by s = 2^-n, n the number of its nonzero exponents (see
    // relax_scaled); *_m multiplies m, *_s sigma, *_a the attractor, *_u the
    // density deviation when the attractor is drho r(a) r(b) r(c). The
    // third-order pairs mix two moments: p3m m_p + p3q m_q + p3s sigma_p +
    // p3t sigma_q.
    R p3m, p3q, p3s, p3t;
    R o3m, o3s;                  // xyz
    R o4am, o4aa, o4au, o4as;    // xxyy-type
    R o4bm, o4bs;                // xxyz-type
    R o5m, o5s;                  // fifth order
    R o6m, o6a, o6u, o6s;        // sixth order
};

// Fill the relaxation coefficients of P from its rates (host or device).
template <typename R>
CM_HD void derive_coefficients(Rates<R>& P) {
    const R A = R(0.5) * (P.w3a + P.w3b), B = R(0.5) * (P.w3a - P.w3b);
    const R q = R(0.25), e = R(0.125);   // scales of 2 and 3 nonzero exponents
    P.p3m = q * (R(1) - A);
    P.p3q = -q * B;
    P.p3s = q * (R(1) - R(0.5) * A);
    P.p3t = -q * R(0.5) * B;
    P.o3m = e * (R(1) - P.w3c);
    P.o3s = e * (R(1) - R(0.5) * P.w3c);
    P.o4am = q * (R(1) - P.w4a);
    P.o4aa = q * P.w4a;
    P.o4au = q * P.w4a * (R(1) / R(9));
    P.o4as = q * (R(1) - R(0.5) * P.w4a);
    P.o4bm = e * (R(1) - P.w4b);
    P.o4bs = e * (R(1) - R(0.5) * P.w4b);
    P.o5m = e * (R(1) - P.w5);
    P.o5s = e * (R(1) - R(0.5) * P.w5);
    P.o6m = e * (R(1) - P.w6);
    P.o6a = e * P.w6;
    P.o6u = e * P.w6 * (R(1) / R(27));
    P.o6s = e * (R(1) - R(0.5) * P.w6);
}

// ------------------------------------------------------------ source moments
// Central moments sigma of the source (exact identity of the paper: the
// central moment (a,b,c) of the force term is a F_x/rho kappa_{a-1,b,c} +
// b F_y/rho kappa_{a,b-1,c} + c F_z/rho kappa_{a,b,c-1}), with the moments of
// the untransformed f recovered order by order as kappa = kappabar + sigma/2.
// kappa_1 = 0 for the conserved moments, so every second-order sigma vanishes
// and the sweep starts at order three. On return sig[p] holds sigma for
// orders >= 3 (zero below) and kap[p] the full kappa for orders 2..5.
template <typename R>
CM_HD void source_moments(const R (&m)[27], R fx, R fy, R fz, R rho0, R (&sig)[27], R (&kap)[27]) {
    const R f[3] = {fx, fy, fz};
#pragma unroll
    for (int p = 0; p < 27; ++p) {
        sig[p] = R(0);
        kap[p] = ord(p) == 2 ? plus_rest(m[p], rho0, p) : R(0);
    }
#pragma unroll
    for (int k = 0; k < 17; ++k) {
        const int p = high(k);
        R s = R(0);
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (ex_(p, d) > 0) s += R(ex_(p, d)) * f[d] * kap[lower(p, d)];
        sig[p] = s;
        if (ord(p) < 6) kap[p] = plus_rest(m[p], rho0, p) + R(0.5) * s;
    }
}

// ------------------------------------------------------------ eddy viscosity
// Smagorinsky shear rate from the traceless second-order central moments
// (project addition; uses nu = cs^2 (1/omega - 1/2)):
// tau_eff = (tau0 + sqrt(tau0^2 + 18 Cs^2 Q / rho)) / 2, Q = sqrt(2 Pi^d : Pi^d).
template <typename R, bool FAST = false>
CM_HD R eddy_rate(const R (&m)[27], R inv_rho, const Rates<R>& P) {
    const R xx = m[I(2, 0, 0)], yy = m[I(0, 2, 0)], zz = m[I(0, 0, 2)];
    const R tr = (xx + yy + zz) * (R(1) / R(3));
    const R dxx = xx - tr, dyy = yy - tr, dzz = zz - tr;
    const R xy = m[I(1, 1, 0)], xz = m[I(1, 0, 1)], yz = m[I(0, 1, 1)];
    const R pp = dxx * dxx + dyy * dyy + dzz * dzz + R(2) * (xy * xy + xz * xz + yz * yz);
    const R q = sqrt_<FAST>(R(2) * pp);
    const R tau = R(0.5) * (P.tau0 + sqrt_<FAST>(P.tau0 * P.tau0 + P.smag * q * inv_rho));
    return rcp_<FAST>(tau);
}

// ------------------------------------------------------------ relaxation
// v <- R v on the moments of order >= 2 (group rates; R is symmetric).
// Orders 0 and 1 are left untouched.
template <typename R>
CM_HD void apply_rates(R (&v)[27], R ws, const Rates<R>& P) {
    const R third = R(1) / R(3), half = R(0.5);
    {
        const R t = (v[I(2, 0, 0)] + v[I(0, 2, 0)] + v[I(0, 0, 2)]) * third * (P.wb - ws);
        v[I(2, 0, 0)] = ws * v[I(2, 0, 0)] + t;
        v[I(0, 2, 0)] = ws * v[I(0, 2, 0)] + t;
        v[I(0, 0, 2)] = ws * v[I(0, 0, 2)] + t;
        v[I(1, 1, 0)] *= ws;
        v[I(1, 0, 1)] *= ws;
        v[I(0, 1, 1)] *= ws;
    }
    auto pair = [&](int p, int q) {
        const R a = P.w3a * (v[p] + v[q]), b = P.w3b * (v[p] - v[q]);
        v[p] = half * (a + b);
        v[q] = half * (a - b);
    };
    pair(I(1, 2, 0), I(1, 0, 2));
    pair(I(2, 1, 0), I(0, 1, 2));
    pair(I(2, 0, 1), I(0, 2, 1));
    v[I(1, 1, 1)] *= P.w3c;
    v[I(2, 2, 0)] *= P.w4a;
    v[I(2, 0, 2)] *= P.w4a;
    v[I(0, 2, 2)] *= P.w4a;
    v[I(2, 1, 1)] *= P.w4b;
    v[I(1, 2, 1)] *= P.w4b;
    v[I(1, 1, 2)] *= P.w4b;
    v[I(2, 2, 1)] *= P.w5;
    v[I(2, 1, 2)] *= P.w5;
    v[I(1, 2, 2)] *= P.w5;
    v[I(2, 2, 2)] *= P.w6;
}

// m <- m + R d + sigma on the moments of order >= 2, R the group rates of
// apply_rates, written with explicit fused multiply-adds (the build fuses only
// within an expression). sigma vanishes at second order.
template <typename R>
CM_HD void relax_update(R (&m)[27], const R (&d)[27], const R (&sig)[27], R ws, const Rates<R>& P) {
    const R t = (d[I(2, 0, 0)] + d[I(0, 2, 0)] + d[I(0, 0, 2)]) * (R(1) / R(3)) * (P.wb - ws);
    m[I(2, 0, 0)] += fmad(ws, d[I(2, 0, 0)], t);
    m[I(0, 2, 0)] += fmad(ws, d[I(0, 2, 0)], t);
    m[I(0, 0, 2)] += fmad(ws, d[I(0, 0, 2)], t);
    m[I(1, 1, 0)] = fmad(ws, d[I(1, 1, 0)], m[I(1, 1, 0)]);
    m[I(1, 0, 1)] = fmad(ws, d[I(1, 0, 1)], m[I(1, 0, 1)]);
    m[I(0, 1, 1)] = fmad(ws, d[I(0, 1, 1)], m[I(0, 1, 1)]);
    const R ha = R(0.5) * P.w3a, hb = R(0.5) * P.w3b;
    auto pair = [&](int p, int q) {
        const R sp = d[p] + d[q], dm = d[p] - d[q];
        m[p] = fmad(ha, sp, fmad(hb, dm, m[p] + sig[p]));
        m[q] = fmad(ha, sp, fmad(-hb, dm, m[q] + sig[q]));
    };
    pair(I(1, 2, 0), I(1, 0, 2));
    pair(I(2, 1, 0), I(0, 1, 2));
    pair(I(2, 0, 1), I(0, 2, 1));
    auto one = [&](int p, R w) { m[p] = fmad(w, d[p], m[p] + sig[p]); };
    one(I(1, 1, 1), P.w3c);
    one(I(2, 2, 0), P.w4a);
    one(I(2, 0, 2), P.w4a);
    one(I(0, 2, 2), P.w4a);
    one(I(2, 1, 1), P.w4b);
    one(I(1, 2, 1), P.w4b);
    one(I(1, 1, 2), P.w4b);
    one(I(2, 2, 1), P.w5);
    one(I(2, 1, 2), P.w5);
    one(I(1, 2, 2), P.w5);
    one(I(2, 2, 2), P.w6);
}

// Relaxation of the non-conserved central moments towards the attractor
// kappabar^M = kappa^M - sigma/2 (in deviation variables drho r(a)r(b)r(c) -
// sigma/2) with the group rates, plus the source moments sigma; conserved
// moments take their post-collision values (drho, kappabar_1 + F).
// VAR enables the run-time variants: with P.fact the even fourth- and
// sixth-order attractors are the Cartesian products of the post-collision
// second-order central moments divided by rho per extra factor (Sec. 13),
// written in deviation form; with P.rc the first-order central moments of
// fbar are -drho u - F/2 instead of -F/2 (Sec. 12).
template <typename R, bool VAR = false, bool FAST = false>
CM_HD void relax(R (&m)[27], const R (&sig)[27], R drho, R Fx, R Fy, R Fz, R ws, const Rates<R>& P) {
    R d[27];
#pragma unroll
    for (int p = 0; p < 27; ++p) {
        // drho r(a)r(b)r(c) - sigma/2 - m, with the terms that vanish for this
        // moment left out (sigma is zero at second order, r(1) = 0)
        const R u = unit27<R>(p);
        if (ord(p) < 2) d[p] = R(0);
        else if (ord(p) == 2) d[p] = u != R(0) ? fmad(drho, u, -m[p]) : -m[p];
        else d[p] = u != R(0) ? fmad(drho, u, fmad(R(-0.5), sig[p], -m[p])) : fmad(R(-0.5), sig[p], -m[p]);
    }
    if constexpr (VAR) {
        if (P.fact) {
            const R third = R(1) / R(3);
            const R t = (d[I(2, 0, 0)] + d[I(0, 2, 0)] + d[I(0, 0, 2)]) * third * (P.wb - ws);
            const R qx = m[I(2, 0, 0)] + ws * d[I(2, 0, 0)] + t;   // post-collision deviations of xx, yy, zz
            const R qy = m[I(0, 2, 0)] + ws * d[I(0, 2, 0)] + t;
            const R qz = m[I(0, 0, 2)] + ws * d[I(0, 0, 2)] + t;
            const R r0 = P.rho0;
            const R inv = rcp_<FAST>(r0 + drho);
            const R a0 = -r0 * drho * (R(1) / R(9));
            const R axy = (a0 + r0 * third * (qx + qy) + qx * qy) * inv;
            const R axz = (a0 + r0 * third * (qx + qz) + qx * qz) * inv;
            const R ayz = (a0 + r0 * third * (qy + qz) + qy * qz) * inv;
            const R axyz = (-r0 * drho * (r0 + r0 + drho) * (R(1) / R(27)) + r0 * r0 * (R(1) / R(9)) * (qx + qy + qz) +
                            r0 * third * (qx * qy + qx * qz + qy * qz) + qx * qy * qz) *
                           inv * inv;
            d[I(2, 2, 0)] = axy - R(0.5) * sig[I(2, 2, 0)] - m[I(2, 2, 0)];
            d[I(2, 0, 2)] = axz - R(0.5) * sig[I(2, 0, 2)] - m[I(2, 0, 2)];
            d[I(0, 2, 2)] = ayz - R(0.5) * sig[I(0, 2, 2)] - m[I(0, 2, 2)];
            d[I(2, 2, 2)] = axyz - R(0.5) * sig[I(2, 2, 2)] - m[I(2, 2, 2)];
        }
    }
    relax_update(m, d, sig, ws, P);
    bool rc = false;
    if constexpr (VAR) rc = P.rc != 0;
    if (rc) {
        m[I(1, 0, 0)] += Fx;
        m[I(0, 1, 0)] += Fy;
        m[I(0, 0, 1)] += Fz;
    } else {
        m[I(1, 0, 0)] = R(0.5) * Fx;
        m[I(0, 1, 0)] = R(0.5) * Fy;
        m[I(0, 0, 1)] = R(0.5) * Fz;
    }
}

// Density deviation and momentum sum_i h_i e_i of deviation populations.
template <typename R>
CM_HD void mass_momentum(const R (&h)[27], R& drho, R& jx, R& jy, R& jz) {
    R pz[3], py[3], px[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) { pz[k] = R(0); py[k] = R(0); px[k] = R(0); }
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        pz[i / 9] += h[i];
        py[(i / 3) % 3] += h[i];
        px[i % 3] += h[i];
    }
    drho = pz[0] + pz[1] + pz[2];
    jx = px[2] - px[0];
    jy = py[2] - py[0];
    jz = pz[2] - pz[0];
}

// ------------------------------------------------------------ sub-grid stress
// Smagorinsky stress from the pre-collision central moments (Sec. 14
// coupling): with S = -omega0 Pi^d / (2 rho cs^2) and R^d = -2 C_s^2 |S| S,
// R^d = sgs Q Pi^d / rho^2, Q = sqrt(2 Pi^d : Pi^d), sgs = C_s^2 omega0^2 / (2 cs^4).
// Output order: xx, yy, zz, xy, xz, yz.
template <typename R, bool FAST = false>
CM_HD void sgs_stress(const R (&m)[27], R inv_rho, const Rates<R>& P, R (&st)[6]) {
    const R xx = m[I(2, 0, 0)], yy = m[I(0, 2, 0)], zz = m[I(0, 0, 2)];
    const R tr = (xx + yy + zz) * (R(1) / R(3));
    const R dxx = xx - tr, dyy = yy - tr, dzz = zz - tr;
    const R xy = m[I(1, 1, 0)], xz = m[I(1, 0, 1)], yz = m[I(0, 1, 1)];
    const R pp = dxx * dxx + dyy * dyy + dzz * dzz + R(2) * (xy * xy + xz * xz + yz * yz);
    const R c = P.sgs * sqrt_<FAST>(R(2) * pp) * inv_rho * inv_rho;
    st[0] = c * dxx;
    st[1] = c * dyy;
    st[2] = c * dzz;
    st[3] = c * xy;
    st[4] = c * xz;
    st[5] = c * yz;
}

// ------------------------------------------------------------ collision, one line at a time
// The collision of collide_lines takes the frame change of Eq. binomialtheorem
// in two steps per axis: raw moments first (the three-point sums, which need no
// velocity and give the density and momentum on the way), then the shift of
// every axis line to the central moments about u; back to velocity space the
// same in reverse. Each step acts on the lines of one axis only, so the axes
// can be taken in any order.

// Raw moments along one axis: values at e = -1, 0, +1 -> sum, first, second.
template <typename R>
CM_HD void raw3(R& a, R& b, R& c) {
    const R s = a + c;
    const R d = c - a;
    a = s + b;
    b = d;
    c = s;
}

// Raw moments (deviations) -> central moments about u along one axis; rho0 cK
// is the rest-state zeroth moment of the line (cK the unit Maxwellian moments
// of its other two exponents, a compile-time constant).
template <typename R>
CM_HD void shift3(R& m0, R& m1, R& m2, R u, R rho0, R cK) {
    const R kf = cK == R(0) ? m0 : m0 + rho0 * cK;
    const R k1 = m1 - u * kf;
    m2 = m2 - u * (m1 + k1);   // m2 - 2 u m1 + u^2 kf
    m1 = k1;
}

// Central -> raw moments along one axis for moments kept scaled: the entries of
// order 1 and 2 along this axis carry an extra factor 1/2 (k1h, k2h), so that
// the return to populations needs no halving; hu = u/2, rho0 cK the
// rest-state zeroth moment of the line at the line's scale (cK a compile-time
// constant).
template <typename R>
CM_HD void unshift3h(R& k0, R& k1h, R& k2h, R u, R hu, R rho0, R cK) {
    const R kf = cK == R(0) ? k0 : k0 + rho0 * cK;
    const R m1h = k1h + hu * kf;
    k2h = k2h + u * (k1h + m1h);   // (k2 + 2 u k1 + u^2 kf) / 2
    k1h = m1h;
}

// Scaled raw moments (m0, m1/2, m2/2) -> values at e = -1, 0, +1.
template <typename R>
CM_HD void pop3h(R& m0, R& m1h, R& m2h) {
    const R fm = m2h - m1h;
    const R f0 = m0 - R(2) * m2h;
    const R fp = m2h + m1h;
    m0 = fm;
    m1h = f0;
    m2h = fp;
}

// Rest-state zeroth moment factor of a line whose other two exponents are a
// and b, at the line's scale: unit Maxwellian moment r(e) = 1, 0, 1/3 times
// the scale 1, 1/2, 1/2 of each exponent.
template <typename R> CM_HD constexpr R ks1(int e) { return e == 0 ? R(1) : (e == 1 ? R(0) : R(1) / R(6)); }

// Post-collision central moments, written scaled by 2^-n (n the number of
// nonzero exponents of each moment), from the pre-collision ones: the
// relaxation of `relax` (the same attractors, rates and groups) in closed form,
// (1 - R) m + R a + (1 - R/2) sigma per group, with the coefficients of
// derive_coefficients for the orders >= 3.
template <typename R, bool VAR = false, bool FAST = false>
CM_HD void relax_scaled(R (&m)[27], const R (&sig)[27], R drho, R Fx, R Fy, R Fz, R ws, const Rates<R>& P) {
    const R mxx = m[I(2, 0, 0)], myy = m[I(0, 2, 0)], mzz = m[I(0, 0, 2)];
    // second order: deviatoric part with ws, trace with wb; attractor drho/3 for
    // xx, yy, zz and 0 for xy, xz, yz; the trace correction t = (wb - ws)/3
    // (drho - mxx - myy - mzz)
    const R c1 = R(1) - ws;
    const R th = (P.wb - ws) * (R(1) / R(6)) * (drho - (mxx + myy + mzz));   // t / 2
    const R base = ws * (drho * (R(1) / R(6))) + th;                          // (ws drho/3 + t) / 2
    const R c1h = R(0.5) * c1, c1q = R(0.25) * c1;
    m[I(2, 0, 0)] = c1h * mxx + base;
    m[I(0, 2, 0)] = c1h * myy + base;
    m[I(0, 0, 2)] = c1h * mzz + base;
    m[I(1, 1, 0)] *= c1q;
    m[I(1, 0, 1)] *= c1q;
    m[I(0, 1, 1)] *= c1q;
    // third order: (xyy, xzz), (xxy, yzz), (xxz, yyz) relax their sum with w3a
    // and difference with w3b (attractors 0)
    auto pair = [&](int p, int q) {
        const R mp = m[p], mq = m[q];
        m[p] = P.p3m * mp + (P.p3q * mq + (P.p3s * sig[p] + P.p3t * sig[q]));
        m[q] = P.p3m * mq + (P.p3q * mp + (P.p3s * sig[q] + P.p3t * sig[p]));
    };
    pair(I(1, 2, 0), I(1, 0, 2));
    pair(I(2, 1, 0), I(0, 1, 2));
    pair(I(2, 0, 1), I(0, 2, 1));
    auto zero_att = [&](int p, R cm, R cs) { m[p] = cm * m[p] + cs * sig[p]; };
    zero_att(I(1, 1, 1), P.o3m, P.o3s);
    zero_att(I(2, 1, 1), P.o4bm, P.o4bs);
    zero_att(I(1, 2, 1), P.o4bm, P.o4bs);
    zero_att(I(1, 1, 2), P.o4bm, P.o4bs);
    zero_att(I(2, 2, 1), P.o5m, P.o5s);
    zero_att(I(2, 1, 2), P.o5m, P.o5s);
    zero_att(I(1, 2, 2), P.o5m, P.o5s);
    bool fact = false;
    if constexpr (VAR) fact = P.fact != 0;
    if (fact) {
        // factorized attractors (Sec. 13): products of the post-collision
        // second-order central moments (unscaled deviations qx, qy, qz)
        const R third = R(1) / R(3);
        const R qx = R(2) * m[I(2, 0, 0)], qy = R(2) * m[I(0, 2, 0)], qz = R(2) * m[I(0, 0, 2)];
        const R r0 = P.rho0;
        const R inv = rcp_<FAST>(r0 + drho);
        const R a0 = -r0 * drho * (R(1) / R(9));
        const R axy = (a0 + r0 * third * (qx + qy) + qx * qy) * inv;
        const R axz = (a0 + r0 * third * (qx + qz) + qx * qz) * inv;
        const R ayz = (a0 + r0 * third * (qy + qz) + qy * qz) * inv;
        const R axyz = (-r0 * drho * (r0 + r0 + drho) * (R(1) / R(27)) + r0 * r0 * (R(1) / R(9)) * (qx + qy + qz) +
                        r0 * third * (qx * qy + qx * qz + qy * qz) + qx * qy * qz) *
                       inv * inv;
        m[I(2, 2, 0)] = P.o4am * m[I(2, 2, 0)] + (P.o4aa * axy + P.o4as * sig[I(2, 2, 0)]);
        m[I(2, 0, 2)] = P.o4am * m[I(2, 0, 2)] + (P.o4aa * axz + P.o4as * sig[I(2, 0, 2)]);
        m[I(0, 2, 2)] = P.o4am * m[I(0, 2, 2)] + (P.o4aa * ayz + P.o4as * sig[I(0, 2, 2)]);
        m[I(2, 2, 2)] = P.o6m * m[I(2, 2, 2)] + (P.o6a * axyz + P.o6s * sig[I(2, 2, 2)]);
    } else {
        m[I(2, 2, 0)] = P.o4am * m[I(2, 2, 0)] + (P.o4au * drho + P.o4as * sig[I(2, 2, 0)]);
        m[I(2, 0, 2)] = P.o4am * m[I(2, 0, 2)] + (P.o4au * drho + P.o4as * sig[I(2, 0, 2)]);
        m[I(0, 2, 2)] = P.o4am * m[I(0, 2, 2)] + (P.o4au * drho + P.o4as * sig[I(0, 2, 2)]);
        m[I(2, 2, 2)] = P.o6m * m[I(2, 2, 2)] + (P.o6u * drho + P.o6s * sig[I(2, 2, 2)]);
    }
    // conserved moments (scale 1/2 for the first order): drho stays; the first
    // central moments of fbar become +F/2 (or, with reduced compressibility,
    // gain F)
    bool rc = false;
    if constexpr (VAR) rc = P.rc != 0;
    if (rc) {
        m[I(1, 0, 0)] = R(0.5) * (m[I(1, 0, 0)] + Fx);
        m[I(0, 1, 0)] = R(0.5) * (m[I(0, 1, 0)] + Fy);
        m[I(0, 0, 1)] = R(0.5) * (m[I(0, 0, 1)] + Fz);
    } else {
        m[I(1, 0, 0)] = R(0.25) * Fx;
        m[I(0, 1, 0)] = R(0.25) * Fy;
        m[I(0, 0, 1)] = R(0.25) * Fz;
    }
}

// ------------------------------------------------------------ collision
// h: deviation populations (fbar - rho0 w) in, post-collision deviations out.
// rho and u (pre-collision, time n) are returned. The raw moments (three-point
// sums by axis) give the density and momentum before the frame change to the
// central moments needs the velocity.
// SGS (Sec. 14 coupling): the force is F + rho acc (acc = -div R of the
// previous step) and the sub-grid stress of this step is returned in st.
// collide_lines: the same, starting from the velocity-independent sums of the
// nine z-lines (ix, iy) = (l % 3, l / 3) of populations a = h[l], b = h[l + 9],
// c = h[l + 18]: ls[l] = a + c, ld[l] = c - a and h[l] = ls[l] + b (h[9..26]
// are outputs only). Callers holding the populations in another form (FP16
// pairs) form these sums themselves.
template <typename R, bool LES, bool VAR = false, bool SGS = false, bool FAST = false>
CM_HD void collide_lines(R (&h)[27], const R (&ls)[9], const R (&ld)[9], R Fx, R Fy, R Fz, const Rates<R>& P,
                         R& rho_out, R& ux_out, R& uy_out, R& uz_out, const R* acc = nullptr, R* st = nullptr) {
    // raw moments: the z-line sums given, then the y and x lines
#pragma unroll
    for (int l = 0; l < 9; ++l) {
        h[l + 9] = ld[l];
        h[l + 18] = ls[l];
    }
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) {
            const int b = ix + 9 * cz;
            raw3(h[b], h[b + 3], h[b + 6]);
        }
#pragma unroll
    for (int k = 0; k < 9; ++k) raw3(h[3 * k], h[3 * k + 1], h[3 * k + 2]);
    const R drho = h[I(0, 0, 0)], jx = h[I(1, 0, 0)], jy = h[I(0, 1, 0)], jz = h[I(0, 0, 1)];
    const R rho = P.rho0 + drho;
    const R inv_rho = rcp_<FAST>(rho);
    R inv_rho_u = inv_rho;   // density in the momentum: rho, or rho0 with reduced compressibility
    if constexpr (VAR) inv_rho_u = P.rc ? R(1) / P.rho0 : inv_rho;
    if constexpr (SGS) {
        Fx += rho * acc[0];
        Fy += rho * acc[1];
        Fz += rho * acc[2];
    }
    const R ux = (jx + R(0.5) * Fx) * inv_rho_u;
    const R uy = (jy + R(0.5) * Fy) * inv_rho_u;
    const R uz = (jz + R(0.5) * Fz) * inv_rho_u;
    // central moments about u, axis by axis
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int cy = 0; cy < 3; ++cy) {
            const int b = 3 * cy + 9 * cz;
            shift3(h[b], h[b + 1], h[b + 2], ux, P.rho0, r1<R>(cy) * r1<R>(cz));
        }
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int cx = 0; cx < 3; ++cx) {
            const int b = cx + 9 * cz;
            shift3(h[b], h[b + 3], h[b + 6], uy, P.rho0, r1<R>(cx) * r1<R>(cz));
        }
#pragma unroll
    for (int b = 0; b < 9; ++b) shift3(h[b], h[b + 9], h[b + 18], uz, P.rho0, r1<R>(b % 3) * r1<R>(b / 3));
    R sig[27], kap[27];
    source_moments(h, Fx * inv_rho, Fy * inv_rho, Fz * inv_rho, P.rho0, sig, kap);
    R ws = P.ws;
    if constexpr (LES) ws = eddy_rate<R, FAST>(h, inv_rho_u, P);
    if constexpr (SGS) {
        R t6[6];
        sgs_stress<R, FAST>(h, inv_rho_u, P, t6);
#pragma unroll
        for (int k = 0; k < 6; ++k) st[k] = t6[k];
    }
    relax_scaled<R, VAR, FAST>(h, sig, drho, Fx, Fy, Fz, ws, P);
    // back to raw moments (scaled) and to populations
    const R hx = R(0.5) * ux, hy = R(0.5) * uy, hz = R(0.5) * uz;
#pragma unroll
    for (int b = 0; b < 9; ++b) unshift3h(h[b], h[b + 9], h[b + 18], uz, hz, P.rho0, ks1<R>(b % 3) * ks1<R>(b / 3));
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int cx = 0; cx < 3; ++cx) {
            const int b = cx + 9 * cz;
            unshift3h(h[b], h[b + 3], h[b + 6], uy, hy, P.rho0, ks1<R>(cx) * ks1<R>(cz));
        }
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int cy = 0; cy < 3; ++cy) {
            const int b = 3 * cy + 9 * cz;
            unshift3h(h[b], h[b + 1], h[b + 2], ux, hx, P.rho0, ks1<R>(cy) * ks1<R>(cz));
        }
#pragma unroll
    for (int k = 0; k < 9; ++k) pop3h(h[3 * k], h[3 * k + 1], h[3 * k + 2]);
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) {
            const int b = ix + 9 * cz;
            pop3h(h[b], h[b + 3], h[b + 6]);
        }
#pragma unroll
    for (int b = 0; b < 9; ++b) pop3h(h[b], h[b + 9], h[b + 18]);
    rho_out = rho;
    ux_out = ux;
    uy_out = uy;
    uz_out = uz;
}

// The velocity-independent sums of the nine z-lines that collide_lines starts
// from (h[l] becomes the line's k0).
template <typename R>
CM_HD void zline_sums(R (&h)[27], R (&ls)[9], R (&ld)[9]) {
#pragma unroll
    for (int l = 0; l < 9; ++l) {
        const R a = h[l], b = h[l + 9], c = h[l + 18];
        ls[l] = a + c;
        ld[l] = c - a;
        h[l] = ls[l] + b;   // k0 of the z-line (ix, iy) = l % 3, l / 3
    }
}

template <typename R, bool LES, bool VAR = false, bool SGS = false, bool FAST = false>
CM_HD void collide(R (&h)[27], R Fx, R Fy, R Fz, const Rates<R>& P, R& rho_out, R& ux_out, R& uy_out, R& uz_out,
                   const R* acc = nullptr, R* st = nullptr) {
    R ls[9], ld[9];
    zline_sums(h, ls, ld);
    collide_lines<R, LES, VAR, SGS, FAST>(h, ls, ld, Fx, Fy, Fz, P, rho_out, ux_out, uy_out, uz_out, acc, st);
}

// Canonical populations (deviations) of the forced equilibrium whose central
// moments equal kappabar^M(rho, u, F) = kappa^M - sigma(kappa^M)/2.
template <typename R>
CM_HD void equilibrium(R (&h)[27], R rho, R ux, R uy, R uz, R Fx, R Fy, R Fz, R rho0, bool rc = false) {
    const R drho = rho - rho0;
    const R F[3] = {Fx, Fy, Fz};
    const R u[3] = {ux, uy, uz};
#pragma unroll
    for (int p = 0; p < 27; ++p) {
        // sigma_p on kappa^M = rho r r r: only the axis with exponent 1 contributes
        R sg = R(0);
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (ex_(p, d) == 1) sg += F[d] * unit27<R>(lower(p, d));
        h[p] = drho * unit27<R>(p) - R(0.5) * sg;
    }
    if (rc) {
        // reduced compressibility: rho0 u = sum fbar e + F/2 makes the first
        // central moments of fbar about u equal to -drho u - F/2
#pragma unroll
        for (int d = 0; d < 3; ++d) h[d == 0 ? I(1, 0, 0) : (d == 1 ? I(0, 1, 0) : I(0, 0, 1))] -= drho * u[d];
    }
    inverse_transform(h, ux, uy, uz, rho0);
}

// ------------------------------------------------------------ adjoint
// Reverse mode of `collide` (LES: with the eddy rate of eddy_rate,
// differentiated through its norm Q, whose derivative is taken as 0 where
// Q = 0; VAR: with the reduced-compressibility velocity of Sec. 12 and the
// factorized attractors of Sec. 13 as P.rc and P.fact select): given h
// (pre-collision deviations, as in collide) and lam = dL/dh~ (adjoint of the
// post-collision populations), overwrite lam with dL/dh and add dL/dF to gF.
template <typename R, bool LES = false, bool VAR = false>
CM_HD void collide_adjoint(const R (&h_in)[27], R (&lam)[27], R Fx, R Fy, R Fz, const Rates<R>& P, R (&gF)[3]) {
    // central moments as in collide_lines: raw moments by axis (density and
    // momentum among them), then the shifts about u
    R m[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) m[i] = h_in[i];
#pragma unroll
    for (int l = 0; l < 9; ++l) raw3(m[l], m[l + 9], m[l + 18]);
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) raw3(m[ix + 9 * cz], m[ix + 9 * cz + 3], m[ix + 9 * cz + 6]);
#pragma unroll
    for (int k = 0; k < 9; ++k) raw3(m[3 * k], m[3 * k + 1], m[3 * k + 2]);
    const R drho = m[I(0, 0, 0)], jx = m[I(1, 0, 0)], jy = m[I(0, 1, 0)], jz = m[I(0, 0, 1)];
    const R rho = P.rho0 + drho;
    const R inv_rho = R(1) / rho;
    // density in the momentum: rho, or rho0 with reduced compressibility
    bool rc = false, fact = false;
    if constexpr (VAR) {
        rc = P.rc != 0;
        fact = P.fact != 0;
    }
    const R inv_rho_u = rc ? R(1) / P.rho0 : inv_rho;
    const R u[3] = {(jx + R(0.5) * Fx) * inv_rho_u, (jy + R(0.5) * Fy) * inv_rho_u, (jz + R(0.5) * Fz) * inv_rho_u};
    const R F[3] = {Fx, Fy, Fz};
    const R f[3] = {Fx * inv_rho, Fy * inv_rho, Fz * inv_rho};
#pragma unroll
    for (int k = 0; k < 9; ++k) shift3(m[3 * k], m[3 * k + 1], m[3 * k + 2], u[0], P.rho0, r1<R>(k % 3) * r1<R>(k / 3));
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
        for (int cx = 0; cx < 3; ++cx) {
            const int b = cx + 9 * cz;
            shift3(m[b], m[b + 3], m[b + 6], u[1], P.rho0, r1<R>(cx) * r1<R>(cz));
        }
#pragma unroll
    for (int b = 0; b < 9; ++b) shift3(m[b], m[b + 9], m[b + 18], u[2], P.rho0, r1<R>(b % 3) * r1<R>(b / 3));
    R sig[27], kap[27];
    source_moments(m, f[0], f[1], f[2], P.rho0, sig, kap);
    // the shear rate: omega_shear, or the eddy rate (as in eddy_rate, keeping
    // the traceless diagonal dxx, dyy, dzz, Q and s = sqrt(tau0^2 + smag Q / rho))
    R ws = P.ws, ldx = R(0), ldy = R(0), ldz = R(0), lq = R(0), ls = R(1);
    if constexpr (LES) {
        const R xx = m[I(2, 0, 0)], yy = m[I(0, 2, 0)], zz = m[I(0, 0, 2)];
        const R tr = (xx + yy + zz) * (R(1) / R(3));
        ldx = xx - tr;
        ldy = yy - tr;
        ldz = zz - tr;
        const R xy = m[I(1, 1, 0)], xz = m[I(1, 0, 1)], yz = m[I(0, 1, 1)];
        const R pp = ldx * ldx + ldy * ldy + ldz * ldz + R(2) * (xy * xy + xz * xz + yz * yz);
        lq = sqrt(R(2) * pp);
        ls = sqrt(P.tau0 * P.tau0 + P.smag * lq * inv_rho_u);
        ws = R(1) / (R(0.5) * (P.tau0 + ls));
    }

    // adjoint of the inverse transform: mu~ = T^{-T} lam, and the velocity
    // dependence of T^{-1}: ub_d += sum_p mu~_p p_d kappa~_{p - e_d}
    R ub[3] = {R(0), R(0), R(0)};
    inverse_transform_T(lam, u[0], u[1], u[2]);
    {
        R mt[27];
#pragma unroll
        for (int p = 0; p < 27; ++p) mt[p] = m[p];
        relax<R, VAR>(mt, sig, drho, Fx, Fy, Fz, ws, P);
#pragma unroll
        for (int p = 0; p < 27; ++p) {
#pragma unroll
            for (int d = 0; d < 3; ++d)
                if (ex_(p, d) > 0) {
                    const int q = lower(p, d);
                    ub[d] += lam[p] * R(ex_(p, d)) * plus_rest(mt[q], P.rho0, q);
                }
        }
    }
    // adjoint of the relaxation: m~ = (I - R) m + R (drho r) + (I - R/2) sigma
    // for orders >= 2, m~_0 = m_0, m~_1 = F/2.
    R nu[27];
#pragma unroll
    for (int p = 0; p < 27; ++p) nu[p] = ord(p) >= 2 ? lam[p] : R(0);
    apply_rates(nu, ws, P);
    // first order: m~_1 = F/2, or m_1 + F with reduced compressibility
    const R h1 = rc ? R(1) : R(0.5);
    R gF_[3] = {h1 * lam[I(1, 0, 0)], h1 * lam[I(0, 1, 0)], h1 * lam[I(0, 0, 1)]};
    R drho_b = R(0);
    R sb[27];   // adjoint of sigma (orders >= 3)
    R mb[27];   // adjoint of m
#pragma unroll
    for (int p = 0; p < 27; ++p) {
        // the factorized attractors replace drho r(p) for the all-even moments of order >= 4
        const bool factp = fact && (p == I(2, 2, 0) || p == I(2, 0, 2) || p == I(0, 2, 2) || p == I(2, 2, 2));
        if (ord(p) >= 2 && unit27<R>(p) != R(0) && !factp) drho_b += nu[p] * unit27<R>(p);
        sb[p] = ord(p) >= 3 ? lam[p] - R(0.5) * nu[p] : R(0);
        mb[p] = ord(p) >= 2 ? lam[p] - nu[p] : (ord(p) == 0 ? lam[p] : (rc ? lam[p] : R(0)));
    }
    R wsb_f = R(0);   // adjoint of ws through the factorized attractors
    if constexpr (VAR) {
        if (fact) {
            // as in relax: q = post-collision second-order diagonal deviations,
            // a_xy = (a0 + r0/3 (qx + qy) + qx qy) / rho, a_xyz = (...) / rho^2
            const R third = R(1) / R(3), r0 = P.rho0, inv = R(1) / (r0 + drho);
            const R dx = drho * third - m[I(2, 0, 0)], dy = drho * third - m[I(0, 2, 0)], dz = drho * third - m[I(0, 0, 2)];
            const R dmean = (dx + dy + dz) * third;
            const R tt = dmean * (P.wb - ws);
            const R qx = m[I(2, 0, 0)] + ws * dx + tt, qy = m[I(0, 2, 0)] + ws * dy + tt, qz = m[I(0, 0, 2)] + ws * dz + tt;
            const R a0 = -r0 * drho * (R(1) / R(9));
            const R axy = (a0 + r0 * third * (qx + qy) + qx * qy) * inv;
            const R axz = (a0 + r0 * third * (qx + qz) + qx * qz) * inv;
            const R ayz = (a0 + r0 * third * (qy + qz) + qy * qz) * inv;
            const R axyz = (-r0 * drho * (r0 + r0 + drho) * (R(1) / R(27)) + r0 * r0 * (R(1) / R(9)) * (qx + qy + qz) +
                            r0 * third * (qx * qy + qx * qz + qy * qz) + qx * qy * qz) * inv * inv;
            const R bxy = nu[I(2, 2, 0)], bxz = nu[I(2, 0, 2)], byz = nu[I(0, 2, 2)], bxyz = nu[I(2, 2, 2)];
            const R inv2 = inv * inv, c9 = r0 * r0 * (R(1) / R(9));
            const R qxb = (bxy * (r0 * third + qy) + bxz * (r0 * third + qz)) * inv +
                          bxyz * (c9 + r0 * third * (qy + qz) + qy * qz) * inv2;
            const R qyb = (bxy * (r0 * third + qx) + byz * (r0 * third + qz)) * inv +
                          bxyz * (c9 + r0 * third * (qx + qz) + qx * qz) * inv2;
            const R qzb = (bxz * (r0 * third + qx) + byz * (r0 * third + qy)) * inv +
                          bxyz * (c9 + r0 * third * (qx + qy) + qx * qy) * inv2;
            drho_b += -(bxy + bxz + byz) * r0 * (R(1) / R(9)) * inv - (bxy * axy + bxz * axz + byz * ayz) * inv -
                      bxyz * (R(2) * r0 * (R(1) / R(27)) * inv + R(2) * axyz * inv);
            // q_a = m_aa + ws d_aa + (wb - ws) mean(d), d_aa = drho/3 - m_aa
            const R qs = qxb + qyb + qzb;
            mb[I(2, 0, 0)] += qxb * (R(1) - ws) - (P.wb - ws) * third * qs;
            mb[I(0, 2, 0)] += qyb * (R(1) - ws) - (P.wb - ws) * third * qs;
            mb[I(0, 0, 2)] += qzb * (R(1) - ws) - (P.wb - ws) * third * qs;
            drho_b += P.wb * third * qs;
            wsb_f = qxb * (dx - dmean) + qyb * (dy - dmean) + qzb * (dz - dmean);
        }
    }
    (void)wsb_f;
    if constexpr (LES) {
        // the second-order update m~ = m + R(ws) d (d = attractor - m) moves with
        // ws by the traceless part of d, i.e. by minus the traceless part of m
        const R xy = m[I(1, 1, 0)], xz = m[I(1, 0, 1)], yz = m[I(0, 1, 1)];
        const R wsb = wsb_f - (lam[I(2, 0, 0)] * ldx + lam[I(0, 2, 0)] * ldy + lam[I(0, 0, 2)] * ldz +
                               lam[I(1, 1, 0)] * xy + lam[I(1, 0, 1)] * xz + lam[I(0, 1, 1)] * yz);
        // ws = 1 / tau, tau = (tau0 + s) / 2, s^2 = tau0^2 + smag Q / rho (rho0 with
        // reduced compressibility)
        const R argb = R(0.25) * (-ws * ws * wsb) / ls;
        if (!rc) drho_b -= argb * P.smag * lq * inv_rho * inv_rho;
        // Q = sqrt(2 pp): dQ/dpp = 1 / Q, taken as 0 at Q = 0
        const R ppb = lq > R(0) ? argb * P.smag * inv_rho_u / lq : R(0);
        mb[I(2, 0, 0)] += R(2) * ldx * ppb;
        mb[I(0, 2, 0)] += R(2) * ldy * ppb;
        mb[I(0, 0, 2)] += R(2) * ldz * ppb;
        mb[I(1, 1, 0)] += R(4) * xy * ppb;
        mb[I(1, 0, 1)] += R(4) * xz * ppb;
        mb[I(0, 1, 1)] += R(4) * yz * ppb;
    }
    // adjoint of the source recursion, highest order first
    R fb[3] = {R(0), R(0), R(0)};
    R kb[27];
#pragma unroll
    for (int p = 0; p < 27; ++p) kb[p] = R(0);
#pragma unroll
    for (int k = 16; k >= 0; --k) {
        const int p = high(k);
        // kappa_p = m_p + const + sigma_p / 2 (orders 3..5): route kb into mb and sb
        if (ord(p) < 6) {
            mb[p] += kb[p];
            sb[p] += R(0.5) * kb[p];
        }
        const R s = sb[p];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (ex_(p, d) > 0) {
                const int q = lower(p, d);
                kb[q] += R(ex_(p, d)) * f[d] * s;
                fb[d] += R(ex_(p, d)) * kap[q] * s;
            }
    }
#pragma unroll
    for (int p = 0; p < 27; ++p)
        if (ord(p) == 2) mb[p] += kb[p];
    // velocity dependence of the forward transform: dm/du_d = -N_d kappabar
#pragma unroll
    for (int p = 0; p < 27; ++p) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (ex_(p, d) > 0) {
                const int q = lower(p, d);
                ub[d] -= mb[p] * R(ex_(p, d)) * plus_rest(m[q], P.rho0, q);
            }
    }
    // adjoint of the forward transform with u fixed: lam <- T^T mb
#pragma unroll
    for (int p = 0; p < 27; ++p) lam[p] = mb[p];
    forward_transform_T(lam, u[0], u[1], u[2]);
    // u = (j + F/2) / rho, f = F / rho, rho = rho0 + sum h
    R rho_b = drho_b;
    R jb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        jb[d] = ub[d] * inv_rho_u;
        gF_[d] += R(0.5) * ub[d] * inv_rho_u + fb[d] * inv_rho;
        rho_b -= (rc ? fb[d] * f[d] : ub[d] * u[d] + fb[d] * f[d]) * inv_rho;
        (void)F[d];
    }
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int ix = i % 3 - 1, iy = (i / 3) % 3 - 1, iz = i / 9 - 1;
        lam[i] += rho_b + R(ix) * jb[0] + R(iy) * jb[1] + R(iz) * jb[2];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) gF[d] += gF_[d];
}

}  // namespace cm
