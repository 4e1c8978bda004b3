// Device kernels of the cascaded central-moment LBM on D2Q9 (gfx950), the
// lattice on which the paper derives the scheme (Secs. 2-13).
//
// Same structure as the D3Q27 kernels: pull scheme, buffers hold the
// post-collision, not yet streamed values; internal layout row-interleaved,
// element (i, x, y) at (y * 9 + i) * nx + x, internal index
// i = (ex+1) + 3 (ey+1), opposite 8 - i.
// Arrays exchanged with callers use the paper's velocity order alpha = 0..8:
// rest, (1,0), (0,1), (-1,0), (0,-1), (1,1), (-1,1), (-1,-1), (1,-1)
// (Sec. 2), structure of arrays, cell c = x + nx y; vector fields have two
// planes (x, y).
//
// Walls (project addition) as in 3D: halfway bounce-back at y = -1/2 and
// y = ny - 1/2 with the moving-wall term 2 w_i rho0 (e_i . U) / cs^2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cm_math2d.hpp"
#include "kernels.hpp"
#include "store.hpp"

namespace cm2 {
using cm::Geom;
using cm::LaunchArgs;
using cm::Store;

__device__ __forceinline__ size_t row_base(const Geom& g, int i, int y) {
    return ((size_t)y * 9 + i) * g.nx;
}

template <typename R>
struct Launch {
    Rates2<R> P;
    R F[2];
    R ulo[2], uhi[2];
    const R* rs_prev;   // sub-grid stress of the previous step, or null (read-out kernels)
};

// a' = -div R of the previous step's sub-grid stress at (x, y) (Sec. 14
// coupling): central differences on the periodic grid; planes xx, yy, xy.
template <typename R>
__device__ __forceinline__ void sgs_accel(const R* __restrict__ rs, const Geom g, int x, int y, R (&a)[2]) {
    const size_t N = (size_t)g.N, nx = (size_t)g.nx;
    const size_t r0 = nx * (size_t)y;
    const size_t ryp = nx * (size_t)(y == g.ny - 1 ? 0 : y + 1);
    const size_t rym = nx * (size_t)(y == 0 ? g.ny - 1 : y - 1);
    const uint32_t ox = (uint32_t)x * (uint32_t)sizeof(R);
    const uint32_t oxp = (uint32_t)(x == g.nx - 1 ? 0 : x + 1) * (uint32_t)sizeof(R);
    const uint32_t oxm = (uint32_t)(x == 0 ? g.nx - 1 : x - 1) * (uint32_t)sizeof(R);
    auto at = [&](int k, size_t r, uint32_t o) { return *(const R*)((const char*)(rs + k * N + r) + o); };
    a[0] = R(-0.5) * ((at(0, r0, oxp) - at(0, r0, oxm)) + (at(2, ryp, ox) - at(2, rym, ox)));
    a[1] = R(-0.5) * ((at(2, r0, oxp) - at(2, r0, oxm)) + (at(1, ryp, ox) - at(1, rym, ox)));
}

template <int S, bool NT = false, typename R = typename Store<S>::R>
__device__ __forceinline__ R load_dev(const typename Store<S>::T* p, int i, R rho0) {
    R v;
    if constexpr (NT) v = static_cast<R>(__builtin_nontemporal_load(p));
    else v = static_cast<R>(*p);
    if constexpr (!Store<S>::shifted) v -= rho0 * w9<R>(i);
    return v;
}

template <int S, typename R = typename Store<S>::R>
__device__ __forceinline__ typename Store<S>::T to_store(R v, int i, R rho0) {
    if constexpr (!Store<S>::shifted) v += rho0 * w9<R>(i);
    return static_cast<typename Store<S>::T>(v);
}

template <typename R>
__device__ __forceinline__ R wall_term(int i, const R (&U)[2], R rho0) {
    const int ex = i % 3 - 1, ey = i / 3 - 1;
    return R(6) * w9<R>(i) * rho0 * (R(ex) * U[0] + R(ey) * U[1]);
}

// Gather of fbar(n) at (x, y): y is uniform per block, so the nine source
// rows are uniform pointers and only the x offset varies across lanes.
template <int S, bool WALLS, typename R = typename Store<S>::R>
__device__ __forceinline__ void gather(const typename Store<S>::T* __restrict__ src, const Geom g, int x, int y,
                                       const Launch<R>& L, R (&h)[9]) {
    using T = typename Store<S>::T;
    const uint32_t xo[3] = {(uint32_t)(x == g.nx - 1 ? 0 : x + 1) * (uint32_t)sizeof(T), (uint32_t)x * (uint32_t)sizeof(T),
                            (uint32_t)(x == 0 ? g.nx - 1 : x - 1) * (uint32_t)sizeof(T)};
    const int ys[3] = {y == g.ny - 1 ? 0 : y + 1, y, y == 0 ? g.ny - 1 : y - 1};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int ix = i % 3, iy = i / 3;
        if constexpr (WALLS) {
            const bool from_lo = (iy == 2) && (y == 0);
            const bool from_hi = (iy == 0) && (y == g.ny - 1);
            if (from_lo || from_hi) {
                const int o = 8 - i;
                const T* row = src + row_base(g, o, y);
                R v = load_dev<S, true>((const T*)((const char*)row + xo[1]), o, L.P.rho0);
                v += wall_term<R>(i, from_lo ? L.ulo : L.uhi, L.P.rho0);
                h[i] = v;
                continue;
            }
        }
        const T* row = src + row_base(g, i, ys[iy]);
        // the rows read at x are read once (non-temporal); the x-shifted ones
        // keep ordinary loads, so that the lines a wave shares with its
        // neighbour stay in L2 (8192^2 FP32: 868 -> 836 us per step)
        if (ix == 1) h[i] = load_dev<S, true>((const T*)((const char*)row + xo[1]), i, L.P.rho0);
        else h[i] = load_dev<S>((const T*)((const char*)row + xo[ix]), i, L.P.rho0);
    }
}

template <int S, bool WALLS, typename R = typename Store<S>::R>
__device__ __forceinline__ void scatter(typename Store<S>::T* __restrict__ dst, const Geom g, int x, int y,
                                        const Launch<R>& L, const R (&h)[9]) {
    const int xs[3] = {x == g.nx - 1 ? 0 : x + 1, x, x == 0 ? g.nx - 1 : x - 1};
    const int ys[3] = {y == g.ny - 1 ? 0 : y + 1, y, y == 0 ? g.ny - 1 : y - 1};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int ix = i % 3, iy = i / 3;
        if constexpr (WALLS) {
            const bool from_lo = (iy == 2) && (y == 0);
            const bool from_hi = (iy == 0) && (y == g.ny - 1);
            if (from_lo || from_hi) {
                const int o = 8 - i;
                const R v = h[i] - wall_term<R>(i, from_lo ? L.ulo : L.uhi, L.P.rho0);
                dst[row_base(g, o, y) + x] = to_store<S>(v, o, L.P.rho0);
                continue;
            }
        }
        dst[row_base(g, i, ys[iy]) + xs[ix]] = to_store<S>(h[i], i, L.P.rho0);
    }
}

template <typename R, bool FFIELD>
__device__ __forceinline__ void cell_force(const R* __restrict__ force, const Geom g, size_t c, const Launch<R>& L,
                                           R& Fx, R& Fy) {
    if constexpr (FFIELD) {
        Fx = force[c];
        Fy = force[(size_t)g.N + c];
    } else {
        (void)force; (void)g; (void)c;
        Fx = L.F[0];
        Fy = L.F[1];
    }
}

// ---------------------------------------------------------------- step
template <int S, bool WALLS, bool LES, bool FFIELD, bool VAR, bool SGS = false>
__global__ void __launch_bounds__(256) k2_step(const typename Store<S>::T* __restrict__ src,
                                               typename Store<S>::T* __restrict__ dst,
                                               const typename Store<S>::R* __restrict__ force, const Geom g,
                                               const Launch<typename Store<S>::R> L,
                                               const typename Store<S>::R* __restrict__ rs_prev = nullptr,
                                               typename Store<S>::R* __restrict__ rs_next = nullptr) {
    using R = typename Store<S>::R;
    using T = typename Store<S>::T;
    int bx, y, z;
    cm::block_coords(g.xcd, bx, y, z);
    for (int x = bx * blockDim.x + threadIdx.x; x < g.nx; x += gridDim.x * blockDim.x) {
        R h[9];
        gather<S, WALLS>(src, g, x, y, L, h);
        const size_t row = (size_t)g.nx * (size_t)y;   // uniform
        R Fx, Fy;
        if constexpr (FFIELD) {
            const uint32_t xb = (uint32_t)x * (uint32_t)sizeof(R);
            Fx = *(const R*)((const char*)(force + row) + xb);
            Fy = *(const R*)((const char*)(force + (size_t)g.N + row) + xb);
        } else {
            Fx = L.F[0];
            Fy = L.F[1];
        }
        R rho, ux, uy;
        if constexpr (SGS) {
            R acc[2], st[3];
            sgs_accel(rs_prev, g, x, y, acc);
            collide9<R, false, VAR, true>(h, Fx, Fy, L.P, rho, ux, uy, acc, st);
#pragma unroll
            for (int k = 0; k < 3; ++k) __builtin_nontemporal_store(st[k], rs_next + (size_t)k * g.N + row + x);
        } else {
            collide9<R, LES, VAR>(h, Fx, Fy, L.P, rho, ux, uy);
        }
        const uint32_t xt = (uint32_t)x * (uint32_t)sizeof(T);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            __builtin_nontemporal_store(to_store<S>(h[i], i, L.P.rho0), (T*)((char*)(dst + row_base(g, i, y)) + xt));
    }
}

// ---------------------------------------------------------------- set-up and read-out
template <int S, bool WALLS, bool FFIELD>
__global__ void __launch_bounds__(256) k2_init_equilibrium(typename Store<S>::T* __restrict__ dst,
                                                           const typename Store<S>::R* __restrict__ force,
                                                           const void* __restrict__ rho_in,
                                                           const void* __restrict__ u_in, int dt, const Geom g,
                                                           const Launch<typename Store<S>::R> L) {
    using R = typename Store<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= g.nx) return;
    const size_t c = (size_t)x + (size_t)g.nx * y;
    const R rho = rho_in ? static_cast<R>(cm::as_double(rho_in, dt, c)) : L.P.rho0;
    const R ux = static_cast<R>(cm::as_double(u_in, dt, c));
    const R uy = static_cast<R>(cm::as_double(u_in, dt, (size_t)g.N + c));
    R Fx, Fy;
    cell_force<R, FFIELD>(force, g, c, L, Fx, Fy);
    R h[9];
    equilibrium9(h, rho, ux, uy, Fx, Fy, L.P.rho0, L.P.rc != 0);
    scatter<S, WALLS>(dst, g, x, y, L, h);
}

template <int S, bool WALLS>
__global__ void __launch_bounds__(256) k2_set_populations(typename Store<S>::T* __restrict__ dst,
                                                          const void* __restrict__ f, int dt, const Geom g,
                                                          const Launch<typename Store<S>::R> L) {
    using R = typename Store<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= g.nx) return;
    const size_t c = (size_t)x + (size_t)g.nx * y;
    R h[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const int i = from_paper(a);
        h[i] = static_cast<R>(cm::as_double(f, dt, (size_t)a * g.N + c) - (double)L.P.rho0 * w9<double>(i));
    }
    scatter<S, WALLS>(dst, g, x, y, L, h);
}

// mode 0: canonical populations (paper order) into out0; mode 1: rho into
// out0 and u (2 planes) into out1
template <int S, bool WALLS, bool FFIELD>
__global__ void __launch_bounds__(256) k2_read(const typename Store<S>::T* __restrict__ src,
                                               const typename Store<S>::R* __restrict__ force, void* __restrict__ out0,
                                               void* __restrict__ out1, int dt, int mode, const Geom g,
                                               const Launch<typename Store<S>::R> L) {
    using R = typename Store<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= g.nx) return;
    const size_t c = (size_t)x + (size_t)g.nx * y;
    R h[9];
    gather<S, WALLS>(src, g, x, y, L, h);
    auto put = [&](void* out, size_t k, double v) {
        if (dt == 0) static_cast<double*>(out)[k] = v;
        else static_cast<float*>(out)[k] = static_cast<float>(v);
    };
    if (mode == 0) {
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const int i = from_paper(a);
            put(out0, (size_t)a * g.N + c, (double)h[i] + (double)L.P.rho0 * w9<double>(i));
        }
        return;
    }
    R Fx, Fy;
    cell_force<R, FFIELD>(force, g, c, L, Fx, Fy);
    R drho = R(0), jx = R(0), jy = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        drho += h[i];
        jx += R(i % 3 - 1) * h[i];
        jy += R(i / 3 - 1) * h[i];
    }
    const R rho = L.P.rho0 + drho;
    if (L.rs_prev) {   // sub-grid stress as a force: F + rho a'
        R a[2];
        sgs_accel(L.rs_prev, g, x, y, a);
        Fx += rho * a[0];
        Fy += rho * a[1];
    }
    const R rho_u = L.P.rc ? L.P.rho0 : rho;   // reduced compressibility: rho0 u = j + F/2
    put(out0, c, (double)rho);
    put(out1, c, (double)((jx + R(0.5) * Fx) / rho_u));
    put(out1, (size_t)g.N + c, (double)((jy + R(0.5) * Fy) / rho_u));
}

// Partial sums per workgroup over tiles of one workgroup width along a grid
// row (x chunk fastest, then y): workgroup b of B combines tiles b, b + B, ...
// lane by lane, then reduces over its lanes (see the D3Q27 kernel).
template <int S, bool WALLS, bool FFIELD>
__global__ void __launch_bounds__(256) k2_reduce_partial(const typename Store<S>::T* __restrict__ src,
                                                         const typename Store<S>::R* __restrict__ force,
                                                         double* __restrict__ partial, const Geom g,
                                                         const Launch<typename Store<S>::R> L) {
    using R = typename Store<S>::R;
    const uint32_t gx = (uint32_t)((g.nx + (int)blockDim.x - 1) / (int)blockDim.x);
    const uint64_t ntiles = (uint64_t)gx * (uint64_t)g.ny;
    const uint64_t nblocks = (uint64_t)gridDim.x * gridDim.y;
    const uint64_t b = blockIdx.x + (uint64_t)gridDim.x * blockIdx.y;
    double v[8] = {0, 0, 0, 0, 0, 0, 1.0e300, 0};
    for (uint64_t t = b; t < ntiles; t += nblocks) {
        const int x = (int)(t % gx) * (int)blockDim.x + (int)threadIdx.x;
        const int y = (int)(t / gx);
        if (x >= g.nx) continue;
        const size_t c = (size_t)x + (size_t)g.nx * y;
        R h[9];
        gather<S, WALLS>(src, g, x, y, L, h);
        double drho = 0, jx = 0, jy = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            drho += (double)h[i];
            jx += (double)(i % 3 - 1) * (double)h[i];
            jy += (double)(i / 3 - 1) * (double)h[i];
        }
        R Fx, Fy;
        cell_force<R, FFIELD>(force, g, c, L, Fx, Fy);
        if (L.rs_prev) {   // sub-grid stress as a force: F + rho a' (rho in the compute type)
            R a[2];
            sgs_accel(L.rs_prev, g, x, y, a);
            const R rho_r = L.P.rho0 + (R)drho;
            Fx += rho_r * a[0];
            Fy += rho_r * a[1];
        }
        const double rho = (double)L.P.rho0 + drho;
        const double rho_u = L.P.rc ? (double)L.P.rho0 : rho;
        const double ux = (jx + 0.5 * (double)Fx) / rho_u, uy = (jy + 0.5 * (double)Fy) / rho_u;
        const double u2 = ux * ux + uy * uy;
        const bool bad = !isfinite(rho) || !isfinite(u2);
        double w[8];
        w[0] = bad ? 0.0 : rho;
        w[1] = bad ? 0.0 : rho * ux;
        w[2] = bad ? 0.0 : rho * uy;
        w[3] = 0.0;
        w[4] = bad ? 0.0 : 0.5 * rho * u2;
        w[5] = bad ? 1.0 : 0.0;
        w[6] = bad ? 1.0e300 : rho;
        w[7] = bad ? 0.0 : sqrt(u2);
        cm::combine(v, w);
    }
    cm::block_reduce(v, partial + 8 * b);
}

// ---------------------------------------------------------------- launch helpers
static dim3 grid_for(const Geom& g, int& bx, bool rowloop) {
    bx = g.nx >= 256 ? 256 : (g.nx >= 128 ? 128 : 64);
    return dim3(rowloop ? 1 : (g.nx + bx - 1) / bx, g.ny, 1);
}

template <typename R>
static Launch<R> make_launch(const LaunchArgs& a) {
    Launch<R> L;
    L.P.rho0 = (R)a.rho0;
    L.P.w3 = (R)a.omega_bulk;
    L.P.ws = (R)a.omega_shear;
    L.P.w6 = (R)a.omega3[0];
    L.P.w7 = (R)a.omega3[1];
    L.P.w8 = (R)a.omega4[0];
    L.P.tau0 = (R)(1.0 / a.omega_shear);
    L.P.smag = (R)(18.0 * a.cs_smag * a.cs_smag);
    L.P.fact = (a.flags & 1u) ? 1 : 0;
    L.P.rc = (a.flags & 2u) ? 1 : 0;
    L.P.sgs = (a.flags & 4u) ? (R)(4.5 * a.cs_smag * a.cs_smag * a.omega_shear * a.omega_shear) : R(0);
    L.rs_prev = (a.flags & 4u) ? (const R*)a.stress_prev : nullptr;
    for (int d = 0; d < 2; ++d) {
        L.F[d] = (R)a.force[d];
        L.ulo[d] = (R)a.wall_u_lo[d];
        L.uhi[d] = (R)a.wall_u_hi[d];
    }
    return L;
}

template <int S, bool W, bool LES, bool FF>
static hipError_t step_t(const LaunchArgs& a, const void* src, void* dst) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    const dim3 grid = grid_for(a.g, bx, a.g.rowloop != 0);
    if (a.flags & 3u)
        k2_step<S, W, LES, FF, true><<<grid, bx, 0, (hipStream_t)a.stream>>>((const T*)src, (T*)dst,
                                                                            (const R*)a.force_field, a.g,
                                                                            make_launch<R>(a));
    else
        k2_step<S, W, LES, FF, false><<<grid, bx, 0, (hipStream_t)a.stream>>>((const T*)src, (T*)dst,
                                                                             (const R*)a.force_field, a.g,
                                                                             make_launch<R>(a));
    return hipGetLastError();
}

// Sub-grid stress as a force (periodic lattices, no eddy rate in the collision).
template <int S, bool FF>
static hipError_t step_sgs_t(const LaunchArgs& a, const void* src, void* dst) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    const dim3 grid = grid_for(a.g, bx, a.g.rowloop != 0);
    hipStream_t st = (hipStream_t)a.stream;
    const Launch<R> L = make_launch<R>(a);
    const R* rp = (const R*)a.stress_prev;
    R* rn = (R*)a.stress_next;
    if (a.flags & 3u)
        k2_step<S, false, false, FF, true, true><<<grid, bx, 0, st>>>((const T*)src, (T*)dst, (const R*)a.force_field, a.g, L, rp, rn);
    else
        k2_step<S, false, false, FF, false, true><<<grid, bx, 0, st>>>((const T*)src, (T*)dst, (const R*)a.force_field, a.g, L, rp, rn);
    return hipGetLastError();
}

template <int S, bool W, bool LES>
static hipError_t step_ff(const LaunchArgs& a, const void* src, void* dst) {
    return a.force_field ? step_t<S, W, LES, true>(a, src, dst) : step_t<S, W, LES, false>(a, src, dst);
}
template <int S, bool W>
static hipError_t step_les(const LaunchArgs& a, const void* src, void* dst) {
    return a.cs_smag > 0.0 ? step_ff<S, W, true>(a, src, dst) : step_ff<S, W, false>(a, src, dst);
}
template <int S>
static hipError_t step_w(const LaunchArgs& a, const void* src, void* dst) {
    if (a.flags & 4u) {
        if (a.walls || !a.stress_prev || !a.stress_next) return hipErrorInvalidValue;   // checked by the caller
        return a.force_field ? step_sgs_t<S, true>(a, src, dst) : step_sgs_t<S, false>(a, src, dst);
    }
    return a.walls ? step_les<S, true>(a, src, dst) : step_les<S, false>(a, src, dst);
}

template <int S, bool W, bool FF>
static hipError_t init_t(const LaunchArgs& a, void* dst, const void* rho, const void* u, int dt) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    const dim3 grid = grid_for(a.g, bx, false);
    k2_init_equilibrium<S, W, FF><<<grid, bx, 0, (hipStream_t)a.stream>>>((T*)dst, (const R*)a.force_field, rho, u,
                                                                          dt, a.g, make_launch<R>(a));
    return hipGetLastError();
}
template <int S>
static hipError_t init_s(const LaunchArgs& a, void* dst, const void* rho, const void* u, int dt) {
    if (a.walls)
        return a.force_field ? init_t<S, true, true>(a, dst, rho, u, dt) : init_t<S, true, false>(a, dst, rho, u, dt);
    return a.force_field ? init_t<S, false, true>(a, dst, rho, u, dt) : init_t<S, false, false>(a, dst, rho, u, dt);
}

template <int S, bool W>
static hipError_t setpop_t(const LaunchArgs& a, void* dst, const void* f, int dt) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    const dim3 grid = grid_for(a.g, bx, false);
    k2_set_populations<S, W><<<grid, bx, 0, (hipStream_t)a.stream>>>((T*)dst, f, dt, a.g, make_launch<R>(a));
    return hipGetLastError();
}
template <int S>
static hipError_t setpop_s(const LaunchArgs& a, void* dst, const void* f, int dt) {
    return a.walls ? setpop_t<S, true>(a, dst, f, dt) : setpop_t<S, false>(a, dst, f, dt);
}

template <int S, bool W, bool FF>
static hipError_t read_t(const LaunchArgs& a, const void* src, void* o0, void* o1, int dt, int mode) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    const dim3 grid = grid_for(a.g, bx, false);
    k2_read<S, W, FF><<<grid, bx, 0, (hipStream_t)a.stream>>>((const T*)src, (const R*)a.force_field, o0, o1, dt,
                                                             mode, a.g, make_launch<R>(a));
    return hipGetLastError();
}
template <int S>
static hipError_t read_s(const LaunchArgs& a, const void* src, void* o0, void* o1, int dt, int mode) {
    if (a.walls)
        return a.force_field ? read_t<S, true, true>(a, src, o0, o1, dt, mode) : read_t<S, true, false>(a, src, o0, o1, dt, mode);
    return a.force_field ? read_t<S, false, true>(a, src, o0, o1, dt, mode) : read_t<S, false, false>(a, src, o0, o1, dt, mode);
}

template <int S, bool W, bool FF>
static hipError_t reduce_t(const LaunchArgs& a, const void* src, double* partial, double* out, size_t max_blocks) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    dim3 grid = grid_for(a.g, bx, false);
    const size_t ntiles = (size_t)grid.x * grid.y;
    if (max_blocks && ntiles > max_blocks) grid = dim3((unsigned)max_blocks, 1, 1);
    k2_reduce_partial<S, W, FF><<<grid, bx, 0, (hipStream_t)a.stream>>>((const T*)src, (const R*)a.force_field,
                                                                       partial, a.g, make_launch<R>(a));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return cm::launch_reduce_final(partial, (size_t)grid.x * grid.y, out, a.stream);
}
template <int S>
static hipError_t reduce_s(const LaunchArgs& a, const void* src, double* partial, double* out, size_t mb) {
    if (a.walls)
        return a.force_field ? reduce_t<S, true, true>(a, src, partial, out, mb) : reduce_t<S, true, false>(a, src, partial, out, mb);
    return a.force_field ? reduce_t<S, false, true>(a, src, partial, out, mb) : reduce_t<S, false, false>(a, src, partial, out, mb);
}

#define CM2_DISPATCH_S(fn, ...)                 \
    switch (a.storage) {                         \
        case 0: return fn<0>(__VA_ARGS__);       \
        case 1: return fn<1>(__VA_ARGS__);       \
        case 2: return fn<2>(__VA_ARGS__);       \
        case 3: return fn<3>(__VA_ARGS__);       \
        default: return hipErrorInvalidValue;    \
    }

hipError_t launch_step(const LaunchArgs& a, const void* src, void* dst) { CM2_DISPATCH_S(step_w, a, src, dst) }
hipError_t launch_init_equilibrium(const LaunchArgs& a, void* dst, const void* rho, const void* u, int dt) {
    CM2_DISPATCH_S(init_s, a, dst, rho, u, dt)
}
hipError_t launch_set_populations(const LaunchArgs& a, void* dst, const void* f, int dt) {
    CM2_DISPATCH_S(setpop_s, a, dst, f, dt)
}
hipError_t launch_read(const LaunchArgs& a, const void* src, void* out0, void* out1, int dt, int mode) {
    CM2_DISPATCH_S(read_s, a, src, out0, out1, dt, mode)
}
hipError_t launch_reduce(const LaunchArgs& a, const void* src, double* partial, double* out, size_t max_blocks) {
    CM2_DISPATCH_S(reduce_s, a, src, partial, out, max_blocks)
}

}  // namespace cm2
