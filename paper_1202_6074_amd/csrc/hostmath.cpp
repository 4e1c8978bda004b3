// Host (CPU) build of the per-cell arithmetic in cm_math.hpp and cm_math2d.hpp
// behind a small C
// interface. It lets the tests check the exact arithmetic of the GPU kernels
// on machines without a GPU. Arrays are structure-of-arrays over n cells:
// populations f[i*n + c] (canonical, unshifted), vectors v[d*n + c].
// rates = {rho0, omega_shear, omega_bulk, omega3a, omega3b, omega3c,
//          omega4a, omega4b, omega5, omega6, cs_smag, flags} (flags: bit 0
//          factorized attractors, bit 1 reduced compressibility, bit 2 the
//          sub-grid stress as a force).
// The D2Q9 entries take populations in the paper's velocity order and
// rates2 = {rho0, omega_3, omega_4 = omega_5, omega_6, omega_7, omega_8,
//           cs_smag, flags}.
#include "cm_math.hpp"
#include "cm_math2d.hpp"

namespace {

template <typename R>
cm::Rates<R> rates_from(const double* r) {
    cm::Rates<R> P;
    P.rho0 = (R)r[0];
    P.ws = (R)r[1];
    P.wb = (R)r[2];
    P.w3a = (R)r[3];
    P.w3b = (R)r[4];
    P.w3c = (R)r[5];
    P.w4a = (R)r[6];
    P.w4b = (R)r[7];
    P.w5 = (R)r[8];
    P.w6 = (R)r[9];
    P.tau0 = (R)(1.0 / r[1]);
    P.smag = (R)(18.0 * r[10] * r[10]);
    P.fact = (int)r[11] & 1;
    P.rc = ((int)r[11] & 2) ? 1 : 0;
    P.sgs = ((int)r[11] & 4) ? (R)(4.5 * r[10] * r[10] * r[1] * r[1]) : R(0);
    cm::derive_coefficients(P);
    return P;
}

// Collision with the sub-grid stress as a force (flags bit 2): force F + rho acc,
// returns the stress of this step (6 planes: xx, yy, zz, xy, xz, yz).
template <typename R>
void collide_sgs_n(const R* f, const R* F, const R* acc, const double* rates, long n, R* out, R* stress) {
    const cm::Rates<R> P = rates_from<R>(rates);
    for (long c = 0; c < n; ++c) {
        R h[27];
        for (int i = 0; i < 27; ++i) h[i] = f[i * n + c] - P.rho0 * cm::w27<R>(i);
        R rho, ux, uy, uz, st[6];
        const R a[3] = {acc[c], acc[n + c], acc[2 * n + c]};
        if (P.fact || P.rc)
            cm::collide<R, false, true, true>(h, F[c], F[n + c], F[2 * n + c], P, rho, ux, uy, uz, a, st);
        else
            cm::collide<R, false, false, true>(h, F[c], F[n + c], F[2 * n + c], P, rho, ux, uy, uz, a, st);
        for (int i = 0; i < 27; ++i) out[i * n + c] = h[i] + P.rho0 * cm::w27<R>(i);
        for (int k = 0; k < 6; ++k) stress[k * n + c] = st[k];
    }
}

template <typename R>
void collide_n(const R* f, const R* F, const double* rates, int les, long n, R* out) {
    const cm::Rates<R> P = rates_from<R>(rates);
    for (long c = 0; c < n; ++c) {
        R h[27];
        for (int i = 0; i < 27; ++i) h[i] = f[i * n + c] - P.rho0 * cm::w27<R>(i);
        R rho, ux, uy, uz;
        const bool var = P.fact || P.rc;   // same dispatch as the step kernel
        if (les && var)
            cm::collide<R, true, true>(h, F[c], F[n + c], F[2 * n + c], P, rho, ux, uy, uz);
        else if (les)
            cm::collide<R, true, false>(h, F[c], F[n + c], F[2 * n + c], P, rho, ux, uy, uz);
        else if (var)
            cm::collide<R, false, true>(h, F[c], F[n + c], F[2 * n + c], P, rho, ux, uy, uz);
        else
            cm::collide<R, false, false>(h, F[c], F[n + c], F[2 * n + c], P, rho, ux, uy, uz);
        for (int i = 0; i < 27; ++i) out[i * n + c] = h[i] + P.rho0 * cm::w27<R>(i);
    }
}

template <typename R>
void adjoint_n(const R* f, const R* F, const double* rates, int les, const R* lam_post, long n, R* lam_pre, R* gF) {
    const cm::Rates<R> P = rates_from<R>(rates);
    for (long c = 0; c < n; ++c) {
        R h[27], lam[27];
        for (int i = 0; i < 27; ++i) {
            h[i] = f[i * n + c] - P.rho0 * cm::w27<R>(i);
            lam[i] = lam_post[i * n + c];
        }
        R g[3] = {R(0), R(0), R(0)};
        const bool var = P.fact || P.rc;   // same dispatch as the adjoint kernel
        if (les && var) cm::collide_adjoint<R, true, true>(h, lam, F[c], F[n + c], F[2 * n + c], P, g);
        else if (les) cm::collide_adjoint<R, true, false>(h, lam, F[c], F[n + c], F[2 * n + c], P, g);
        else if (var) cm::collide_adjoint<R, false, true>(h, lam, F[c], F[n + c], F[2 * n + c], P, g);
        else cm::collide_adjoint<R, false, false>(h, lam, F[c], F[n + c], F[2 * n + c], P, g);
        for (int i = 0; i < 27; ++i) lam_pre[i * n + c] = lam[i];
        for (int d = 0; d < 3; ++d) gF[d * n + c] = g[d];
    }
}

template <typename R>
void equilibrium_n(const R* rho, const R* u, const R* F, double rho0, long n, R* out, int rc) {
    for (long c = 0; c < n; ++c) {
        R h[27];
        cm::equilibrium(h, rho[c], u[c], u[n + c], u[2 * n + c], F[c], F[n + c], F[2 * n + c], (R)rho0, rc != 0);
        for (int i = 0; i < 27; ++i) out[i * n + c] = h[i] + (R)rho0 * cm::w27<R>(i);
    }
}

template <typename R>
cm2::Rates2<R> rates2_from(const double* r) {
    cm2::Rates2<R> P;
    P.rho0 = (R)r[0];
    P.w3 = (R)r[1];
    P.ws = (R)r[2];
    P.w6 = (R)r[3];
    P.w7 = (R)r[4];
    P.w8 = (R)r[5];
    P.tau0 = (R)(1.0 / r[2]);
    P.smag = (R)(18.0 * r[6] * r[6]);
    P.fact = (int)r[7] & 1;
    P.rc = ((int)r[7] & 2) ? 1 : 0;
    P.sgs = ((int)r[7] & 4) ? (R)(4.5 * r[6] * r[6] * r[2] * r[2]) : R(0);
    return P;
}

// D2Q9 collision with the sub-grid stress as a force: force F + rho acc, returns
// the stress of this step (3 planes: xx, yy, xy).
template <typename R>
void collide9_sgs_n(const R* f, const R* F, const R* acc, const double* rates, long n, R* out, R* stress) {
    const cm2::Rates2<R> P = rates2_from<R>(rates);
    for (long c = 0; c < n; ++c) {
        R h[9];
        for (int a = 0; a < 9; ++a) {
            const int i = cm2::from_paper(a);
            h[i] = f[a * n + c] - P.rho0 * cm2::w9<R>(i);
        }
        R rho, ux, uy, st[3];
        const R ac[2] = {acc[c], acc[n + c]};
        if (P.fact || P.rc)
            cm2::collide9<R, false, true, true>(h, F[c], F[n + c], P, rho, ux, uy, ac, st);
        else
            cm2::collide9<R, false, false, true>(h, F[c], F[n + c], P, rho, ux, uy, ac, st);
        for (int a = 0; a < 9; ++a) {
            const int i = cm2::from_paper(a);
            out[a * n + c] = h[i] + P.rho0 * cm2::w9<R>(i);
        }
        for (int k = 0; k < 3; ++k) stress[k * n + c] = st[k];
    }
}

template <typename R>
void collide9_n(const R* f, const R* F, const double* rates, int les, long n, R* out) {
    const cm2::Rates2<R> P = rates2_from<R>(rates);
    for (long c = 0; c < n; ++c) {
        R h[9];
        for (int a = 0; a < 9; ++a) {
            const int i = cm2::from_paper(a);
            h[i] = f[a * n + c] - P.rho0 * cm2::w9<R>(i);
        }
        R rho, ux, uy;
        const bool var = P.fact || P.rc;
        if (les && var)
            cm2::collide9<R, true, true>(h, F[c], F[n + c], P, rho, ux, uy);
        else if (les)
            cm2::collide9<R, true, false>(h, F[c], F[n + c], P, rho, ux, uy);
        else if (var)
            cm2::collide9<R, false, true>(h, F[c], F[n + c], P, rho, ux, uy);
        else
            cm2::collide9<R, false, false>(h, F[c], F[n + c], P, rho, ux, uy);
        for (int a = 0; a < 9; ++a) {
            const int i = cm2::from_paper(a);
            out[a * n + c] = h[i] + P.rho0 * cm2::w9<R>(i);
        }
    }
}

}  // namespace

extern "C" {
void cmhost_collide_sgs_f64(const double* f, const double* F, const double* acc, const double* rates, long n,
                            double* out, double* stress) {
    collide_sgs_n<double>(f, F, acc, rates, n, out, stress);
}
void cmhost_collide9_sgs_f64(const double* f, const double* F, const double* acc, const double* rates2, long n,
                             double* out, double* stress) {
    collide9_sgs_n<double>(f, F, acc, rates2, n, out, stress);
}
void cmhost_collide9_f64(const double* f, const double* F, const double* rates2, int les, long n, double* out) {
    collide9_n<double>(f, F, rates2, les, n, out);
}
void cmhost_collide9_f32(const float* f, const float* F, const double* rates2, int les, long n, float* out) {
    collide9_n<float>(f, F, rates2, les, n, out);
}
void cmhost_equilibrium9_f64(const double* rho, const double* u, const double* F, double rho0, long n, double* out,
                             int rc) {
    for (long c = 0; c < n; ++c) {
        double h[9];
        cm2::equilibrium9(h, rho[c], u[c], u[n + c], F[c], F[n + c], rho0, rc != 0);
        for (int a = 0; a < 9; ++a) {
            const int i = cm2::from_paper(a);
            out[a * n + c] = h[i] + rho0 * cm2::w9<double>(i);
        }
    }
}
void cmhost_collide_f64(const double* f, const double* F, const double* rates, int les, long n, double* out) {
    collide_n<double>(f, F, rates, les, n, out);
}
void cmhost_collide_f32(const float* f, const float* F, const double* rates, int les, long n, float* out) {
    collide_n<float>(f, F, rates, les, n, out);
}
void cmhost_adjoint_f64(const double* f, const double* F, const double* rates, int les, const double* lam_post, long n,
                        double* lam_pre, double* gF) {
    adjoint_n<double>(f, F, rates, les, lam_post, n, lam_pre, gF);
}
void cmhost_equilibrium_f64(const double* rho, const double* u, const double* F, double rho0, long n, double* out,
                            int rc) {
    equilibrium_n<double>(rho, u, F, rho0, n, out, rc);
}
}
