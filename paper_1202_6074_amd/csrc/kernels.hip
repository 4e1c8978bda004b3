// Device kernels of the D3Q27 cascaded central-moment LBM (gfx950).
//
// Internal memory layout (row-interleaved structure of arrays): the nx values
// of population i on grid row (y, z) are contiguous, and the 27 population
// rows of one grid row follow each other:
//     element (i, x, y, z) at ((z * ny + y) * 27 + i) * nx + x.
// A cell's 27 writes therefore land in one contiguous 27-row region and its
// gathers in nine contiguous 3-row regions (the three populations with the
// same (ey, ez) are adjacent), which keeps DRAM accesses local; arrays
// exchanged with callers (populations, moments, force, adjoint) use the plain
// structure of arrays, plane i = population i, cell c = x + nx (y + ny z).
//
// The step kernel is a pull scheme: the buffer between steps holds the
// post-collision, not yet streamed values fbar~(n-1); each thread gathers the
// 27 values arriving at its cell (standard streaming, Eq. cascadedstreaming1),
// collides (Eq. cascadedcollision1) and writes the 27 post-collision values
// back at its own cell into the other buffer. Reads come from the rows of the
// neighbour cells at x +- 1 offsets; writes are aligned and coalesced.
//
// Walls (project addition): halfway bounce-back planes at y = -1/2 and
// y = ny - 1/2 with wall velocities U_lo, U_hi. A population whose upstream
// cell lies in a wall is the opposite population of the same cell plus
// 2 w_i rho0 (e_i . U) / cs^2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "cm_math.hpp"
#include "kernels.hpp"
#include "store.hpp"

namespace cm {

// Offset (in elements) of the row of population i at grid row (y, z) in the
// row-interleaved internal layout. (A plain-plane layout, i N + c, measured
// slower in every storage mode, and a run-time choice between the two cost
// the step kernel a third of its scalar and a sixth of its vector
// instructions, so the layout is fixed.)
__device__ __forceinline__ size_t row_base(const Geom& g, int i, int y, int z) {
    const size_t r = (size_t)z * g.ny + y;
    return (r * 27 + i) * g.nx;
}

// Address of an element: a row pointer that is the same for every lane of the
// workgroup, plus the lane's 32-bit byte offset. Every kernel here takes y and
// z from the block index, so its row pointers are workgroup-uniform; read
// through readfirstlane and typed as global memory, each access then takes the
// scalar-base form of the global load and store instructions (base in scalar
// registers, 32-bit lane offset), where the compiler otherwise forms every
// address with 64-bit vector arithmetic, one instruction per access. Only for
// pointers that are uniform across the workgroup.
template <typename T>
using global_ptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ global_ptr<T> at_row(T* row, uint32_t lane_bytes) {
    // readfirstlane returns a signed 32-bit value: each half goes through
    // uint32_t, so that the low half is zero-extended, not sign-extended.
    const uint64_t v = (uint64_t)row;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    const uint64_t u = ((uint64_t)hi << 32) | (uint64_t)lo;
    return (global_ptr<T>)((global_ptr<char>)u + lane_bytes);
}
// SB: the scalar-base form above, for kernels without a loop around the access
// (inside a loop the uniform read cannot be hoisted and costs more than it
// saves); otherwise the plain pointer.
template <bool SB, typename T>
__device__ __forceinline__ auto row_at(T* row, uint32_t lane_bytes) {
    if constexpr (SB) {
        return at_row(row, lane_bytes);
    } else {
        using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
        return (T*)((C*)row + lane_bytes);
    }
}

template <typename R>
struct Launch {
    Rates<R> P;
    R F[3];        // uniform force (used when no field is given)
    R wt_lo[27], wt_hi[27];   // wall terms per direction, lower and upper wall
    const R* rs_prev;   // sub-grid stress of the previous step, or null (read-out kernels)
};

// Acceleration a' = -div R of the sub-grid stress of the previous step at
// (x, y, z) (Sec. 14 coupling): second-order central differences on the
// periodic grid. Stress planes xx, yy, zz, xy, xz, yz, plain structure of
// arrays; y and z are block-uniform, so the row offsets are uniform.
// sgs_load reads the 18 stress values the differences need, sgs_combine forms
// the acceleration from them (two steps, so that a caller can keep the loads
// in flight together with others).
template <typename R, bool SB = false>
__device__ __forceinline__ void sgs_load(const R* __restrict__ rs, const Geom g, int x, int y, int z, R (&v)[18]) {
    const size_t N = (size_t)g.N, nx = (size_t)g.nx;
    const size_t r0 = nx * ((size_t)y + (size_t)g.ny * z);
    const size_t ryp = nx * ((size_t)(y == g.ny - 1 ? 0 : y + 1) + (size_t)g.ny * z);
    const size_t rym = nx * ((size_t)(y == 0 ? g.ny - 1 : y - 1) + (size_t)g.ny * z);
    const size_t rzp = nx * ((size_t)y + (size_t)g.ny * (z == g.nz - 1 ? 0 : z + 1));
    const size_t rzm = nx * ((size_t)y + (size_t)g.ny * (z == 0 ? g.nz - 1 : z - 1));
    // uniform row pointers, per-lane 32-bit byte offsets (x, x + 1, x - 1 with wrap)
    const uint32_t ox = (uint32_t)x * (uint32_t)sizeof(R);
    const uint32_t oxp = (uint32_t)(x == g.nx - 1 ? 0 : x + 1) * (uint32_t)sizeof(R);
    const uint32_t oxm = (uint32_t)(x == 0 ? g.nx - 1 : x - 1) * (uint32_t)sizeof(R);
    auto at = [&](int k, size_t r, uint32_t o) { return *row_at<SB>(rs + k * N + r, o); };
    // x differences of xx, xy, xz; y differences of xy, yy, yz; z differences of xz, yz, zz
    const int kx[3] = {0, 3, 4}, ky[3] = {3, 1, 5}, kz[3] = {4, 5, 2};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v[2 * c] = at(kx[c], r0, oxp);
        v[2 * c + 1] = at(kx[c], r0, oxm);
        v[6 + 2 * c] = at(ky[c], ryp, ox);
        v[6 + 2 * c + 1] = at(ky[c], rym, ox);
        v[12 + 2 * c] = at(kz[c], rzp, ox);
        v[12 + 2 * c + 1] = at(kz[c], rzm, ox);
    }
}
template <typename R>
__device__ __forceinline__ void sgs_combine(const R (&v)[18], R (&a)[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
        a[c] = R(-0.5) * ((v[2 * c] - v[2 * c + 1]) + (v[6 + 2 * c] - v[6 + 2 * c + 1]) + (v[12 + 2 * c] - v[12 + 2 * c + 1]));
}
template <typename R, bool SB = false>
__device__ __forceinline__ void sgs_accel(const R* __restrict__ rs, const Geom g, int x, int y, int z, R (&a)[3]) {
    R v[18];
    sgs_load<R, SB>(rs, g, x, y, z, v);
    sgs_combine(v, a);
}

// Correction added to a bounced population arriving in direction i from a wall
// moving with velocity U, 2 w_i rho0 (e_i . U) / cs^2, precomputed on the host
// (Launch::wt_lo, wt_hi). It is added and removed with explicitly rounded
// operations, so that no code path fuses it differently into neighbouring
// arithmetic: the two-buffer and in-place schemes then agree bit for bit.
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ float sub_rn(float a, float b) { return __fsub_rn(a, b); }
__device__ __forceinline__ double sub_rn(double a, double b) { return __dsub_rn(a, b); }

// Population loads. Every stored population is read exactly once per step, so
// the loads are non-temporal (measured 7 % faster for FP32 at 256^3, neutral
// for FP64; for FP16 1.5 % faster in the LDS kernel at 256^3 and 3.8 % in the
// even in-place step, since the shorter FP16 collision). Rows that lanes
// read shifted by x -+ 1 share cache lines with the neighbouring wave and keep
// ordinary loads where a wave reads them per lane (the odd in-place step: all
// non-temporal measured 13 % slower, the rows at x alone 1 % faster). In the
// LDS kernel every row is read aligned and once: all non-temporal (ordinary
// loads for the 18 rows exchanged through LDS measured 7 % slower).
template <int S, bool NT = true, typename P = const typename Store<S>::T*>
__device__ __forceinline__ typename Store<S>::T load_raw(P p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Stored value of population i -> deviation from the rest state (compute type),
// and back. The rest-state shift of unshifted storage is rounded explicitly, so
// that no kernel fuses it with neighbouring arithmetic differently from another
// (the step kernels of the different streaming schemes agree bit for bit).
template <int S, typename R = typename Store<S>::R>
__device__ __forceinline__ R from_store(typename Store<S>::T t, int i, R rho0) {
    R v = static_cast<R>(t);
    if constexpr (!Store<S>::shifted) v = sub_rn(v, rho0 * w27<R>(i));
    return v;
}

template <int S, bool NT = true, typename R = typename Store<S>::R, typename P = const typename Store<S>::T*>
__device__ __forceinline__ R load_dev(P p, int i, R rho0) {
    return from_store<S>(load_raw<S, NT>(p), i, rho0);
}

template <int S, typename R = typename Store<S>::R>
__device__ __forceinline__ typename Store<S>::T to_store(R v, int i, R rho0) {
    if constexpr (!Store<S>::shifted) v = add_rn(v, rho0 * w27<R>(i));
    // FP16: the FP32 value is rounded to binary16 on its own (round to nearest
    // even). Without this register constraint the compiler folds the
    // conversion into the last arithmetic operation of some values (one
    // rounding instead of two), differently in different kernels; the FP16
    // kernels then would not agree bit for bit.
    if constexpr (S == 3) asm volatile("" : "+v"(v));
    return static_cast<typename Store<S>::T>(v);
}

// Two FP16 values in one 32-bit word (x, x + 1 of a row; lower address in the
// low half) and back.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));

// Sums of FP16 values held in 32-bit registers (H = 0: the low halves, 1: the
// high halves) with an FP32 result: v_fma_mix_f32 widens its FP16 operands
// exactly and rounds a*1 + c once, which is the FP32 sum of the converted
// values, without the conversion instructions.
template <int H>
__device__ __forceinline__ float mix_add(uint32_t a, uint32_t c) {   // a + c
    float r;
    if constexpr (H == 0) asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(c));
    else asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(c));
    return r;
}
template <int H>
__device__ __forceinline__ float mix_sub(uint32_t c, uint32_t a) {   // c - a
    float r;
    if constexpr (H == 0) asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(c), "v"(a));
    else asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(c), "v"(a));
    return r;
}
template <int H>
__device__ __forceinline__ float mix_addf(uint32_t b, float s) {   // b + s, s in FP32
    float r;
    if constexpr (H == 0) asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(b), "v"(s));
    else asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(b), "v"(s));
    return r;
}
// The velocity-independent z-line sums of collide (ls = a + c, ld = c - a,
// k0 = ls + b) of line l from FP16 values a, b, c in the halves H.
template <int H>
__device__ __forceinline__ void mix_line(uint32_t a, uint32_t b, uint32_t c, float& ls, float& ld, float& k0) {
    ls = mix_add<H>(a, c);
    ld = mix_sub<H>(c, a);
    k0 = mix_addf<H>(b, ls);
}
__device__ __forceinline__ uint32_t pack_f16(float a, float b) {
    // each value rounded to binary16 on its own, as to_store<3> does
    asm volatile("" : "+v"(a), "+v"(b));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((float2_t){a, b}, half2_t));
}


// Gather of fbar(n) at cell (x, y, z).
// MODE 0 (two-buffer pull scheme): the buffer holds fbar~(n-1), population i
//   of the upstream cell x - e_i in plane i, or, when that is a wall, plane
//   26 - i of the cell itself plus the wall term.
// MODE 1 (in-place streaming, even parity): fbar_i(x) sits in plane i of x;
//   a population that arrived from a wall is kept without its wall term,
//   which is added here (the same arithmetic as MODE 0).
// MODE 2 (in-place streaming, odd parity): the previous (even) step stored
//   fbar~_i(x) in plane 26 - i of x, so fbar_i(x) is plane 26 - i of x - e_i,
//   or, from a wall, plane i of x plus the wall term.
// y and z are uniform across a block, so the 27 source rows are uniform
// pointers (scalar registers); only the x offset (x - 1, x, x + 1 with wrap)
// varies across lanes, as a 32-bit byte offset.
// NTX: non-temporal loads also for the x-shifted rows (ex != 0). When a row is
// split between workgroups, the cache lines at the split are read by two of
// them, and ordinary loads keep those lines for the second reader (measured
// +4 % for FP32 at 512^3); the step kernel takes ordinary loads there, and
// gather_xlds when one workgroup covers a row. The read-out kernels keep the
// default.
template <int S, bool WALLS, int MODE = 0, bool NTX = true, bool SB = false, typename R = typename Store<S>::R>
__device__ __forceinline__ void gather(const typename Store<S>::T* src, const Geom g, int x, int y, int z,
                                       const Launch<R>& L, R (&h)[27]) {
    using T = typename Store<S>::T;
    if constexpr (MODE == 1) {
        const uint32_t xt = (uint32_t)x * (uint32_t)sizeof(T);
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            h[i] = load_dev<S, MODE != 2>(row_at<SB>(src + row_base(g, i, y, z), xt), i, L.P.rho0);
            if constexpr (WALLS) {
                const int iy = (i / 3) % 3;
                const bool from_lo = (iy == 2) && (y == 0);
                const bool from_hi = (iy == 0) && (y == g.ny - 1);
                if (from_lo || from_hi) h[i] = add_rn(h[i], from_lo ? L.wt_lo[i] : L.wt_hi[i]);
            }
        }
        return;
    }
    const uint32_t xo[3] = {(uint32_t)(x == g.nx - 1 ? 0 : x + 1) * (uint32_t)sizeof(T), (uint32_t)x * (uint32_t)sizeof(T),
                            (uint32_t)(x == 0 ? g.nx - 1 : x - 1) * (uint32_t)sizeof(T)};   // x - ex, ex = -1, 0, +1
    const int ys[3] = {y == g.ny - 1 ? 0 : y + 1, y, y == 0 ? g.ny - 1 : y - 1};
    const int zs[3] = {z == g.nz - 1 ? 0 : z + 1, z, z == 0 ? g.nz - 1 : z - 1};
    // The three populations of a source row that differ only in ex sit in
    // consecutive rows of the interleaved layout, so each of the nine source
    // rows (ey, ez) needs one uniform pointer, and the row-in-group offset is
    // folded into the three per-lane offsets (scalar-register pressure).
    const uint32_t rb = (uint32_t)g.nx * (uint32_t)sizeof(T);
    uint32_t vo[3];
#pragma unroll
    for (int ix = 0; ix < 3; ++ix) vo[ix] = xo[ix] + (uint32_t)(MODE == 2 ? 2 - ix : ix) * rb;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int ix = i % 3, iy = (i / 3) % 3, iz = i / 9;
        if constexpr (WALLS) {
            const bool from_lo = (iy == 2) && (y == 0);
            const bool from_hi = (iy == 0) && (y == g.ny - 1);
            if (from_lo || from_hi) {
                const int o = MODE == 2 ? i : 26 - i;
                const T* row = src + row_base(g, o, y, z);
                R v = load_dev<S, MODE != 2>(row_at<SB>(row, xo[1]), o, L.P.rho0);
                v = add_rn(v, from_lo ? L.wt_lo[i] : L.wt_hi[i]);
                h[i] = v;
                continue;
            }
        }
        const int pl = MODE == 2 ? 26 - i : i;   // w_i = w_{26-i}: the shift is the same
        const T* grp = src + row_base(g, pl - pl % 3, ys[iy], zs[iz]);
        const auto p = row_at<SB>(grp, vo[ix]);
        // rows read at x once: non-temporal; x-shifted rows: non-temporal only with
        // NTX and not in the odd in-place gather (whose shifted reads share lines
        // with the neighbouring wave; its aligned rows non-temporal: 1024 x 512 x
        // 512 FP32 10,930 -> 10,832 us, FP16 shifted 6,038 -> 5,957 us per pair)
        if (ix == 1 || (MODE != 2 && NTX)) h[i] = load_dev<S, true>(p, pl, L.P.rho0);
        else h[i] = load_dev<S, false>(p, pl, L.P.rho0);
    }
}

// Gather in the mode the geometry's streaming state asks for (read-out kernels).
template <int S, bool WALLS, typename R = typename Store<S>::R>
__device__ __forceinline__ void gather_any(const typename Store<S>::T* src, const Geom g, int x, int y, int z,
                                           const Launch<R>& L, R (&h)[27]) {
    if (g.aa == 0) gather<S, WALLS, 0>(src, g, x, y, z, L, h);
    else if (g.aa == 1) gather<S, WALLS, 1>(src, g, x, y, z, L, h);
    else gather<S, WALLS, 2>(src, g, x, y, z, L, h);
}

// Gather of the two-buffer pull scheme for periodic rows when one workgroup
// covers a whole grid row (nx <= blockDim.x, lanes x >= nx idle): every
// population row is read aligned at x, so each wave reads whole cache lines and
// nothing twice, and the values that cross to x + 1 or x - 1 (the 18 rows with
// e_x != 0) are exchanged through LDS. Against per-lane shifted loads, the
// access pattern alone (trivial arithmetic, 256^3 FP32) runs 7 % faster.
// Every lane of the workgroup must call this (it contains a barrier); idle
// lanes load a valid address and fill LDS columns nobody reads. pin() is
// called after all population loads are issued and before the barrier.
template <int S, bool SB, typename Pin>
__device__ __forceinline__ void gather_xlds(const typename Store<S>::T* src, const Geom g, int x, bool act, int y,
                                            int z, typename Store<S>::T (&out)[27], Pin&& pin) {
    using T = typename Store<S>::T;
    __shared__ T sm[18][256];
    const int ys[3] = {y == g.ny - 1 ? 0 : y + 1, y, y == 0 ? g.ny - 1 : y - 1};
    const int zs[3] = {z == g.nz - 1 ? 0 : z + 1, z, z == 0 ? g.nz - 1 : z - 1};
    const uint32_t rb = (uint32_t)g.nx * (uint32_t)sizeof(T);
    const uint32_t xt = (uint32_t)(act ? x : 0) * (uint32_t)sizeof(T);   // idle lanes read x = 0
    T raw[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int ix = i % 3, iy = (i / 3) % 3, iz = i / 9;
        const T* grp = src + row_base(g, i - ix, ys[iy], zs[iz]);
        if constexpr (SB) raw[i] = load_raw<S>(at_row(grp, xt + (uint32_t)ix * rb));
        else raw[i] = load_raw<S>((const T*)((const char*)grp + xt + (uint32_t)ix * rb));
    }
#pragma unroll
    for (int i = 0; i < 27; ++i)
        if (i % 3 != 1) sm[(i / 3) * 2 + (i % 3) / 2][x] = raw[i];
    // The e_x = 0 values (and the caller's other loads, pin()) are used only
    // after the barrier; without these register constraints the compiler issues
    // their loads after it, a second memory round trip.
#pragma unroll
    for (int i = 1; i < 27; i += 3) asm volatile("" : "+v"(raw[i]));
    pin();
    __syncthreads();
    const int xp = x >= g.nx - 1 ? 0 : x + 1, xm = x == 0 ? g.nx - 1 : x - 1;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int ix = i % 3;   // e_x = ix - 1: the value comes from x - e_x
        out[i] = ix == 1 ? raw[i] : sm[(i / 3) * 2 + ix / 2][ix == 0 ? xp : xm];
    }
}

template <typename R, bool FFIELD>
__device__ __forceinline__ void cell_force(const R* __restrict__ force, const Geom g, int c, const Launch<R>& L, R& Fx,
                                           R& Fy, R& Fz) {
    if constexpr (FFIELD) {
        Fx = force[c];
        Fy = force[(size_t)g.N + c];
        Fz = force[2 * (size_t)g.N + c];
    } else {
        (void)force; (void)g; (void)c;
        Fx = L.F[0];
        Fy = L.F[1];
        Fz = L.F[2];
    }
}

// ---------------------------------------------------------------- step
// The collision of one cell after its gather, and the store of its 27
// post-collision values (and, with SGS, of its sub-grid stress).
template <typename R, bool FFIELD, bool SB = false>
__device__ __forceinline__ void row_force(const R* __restrict__ force, const Geom g, const Launch<R>& L, int x, int y,
                                          int z, R (&F)[3]) {
    if constexpr (FFIELD) {
        const size_t row = (size_t)g.nx * ((size_t)y + (size_t)g.ny * z);   // uniform
        const uint32_t xb = (uint32_t)x * (uint32_t)sizeof(R);
#pragma unroll
        for (int d = 0; d < 3; ++d) F[d] = *row_at<SB>(force + (size_t)d * g.N + row, xb);
    } else {
        (void)force; (void)g; (void)x; (void)y; (void)z;
#pragma unroll
        for (int d = 0; d < 3; ++d) F[d] = L.F[d];
    }
}

// h[0..8], ls, ld: the z-line sums of the gathered populations (zline_sums).
template <int S, bool LES, bool VAR, bool SGS, bool SB = false>
__device__ __forceinline__ void finish_cell(typename Store<S>::T* __restrict__ dst, const Geom g,
                                            const Launch<typename Store<S>::R>& L, int x, int y, int z,
                                            typename Store<S>::R (&h)[27], const typename Store<S>::R (&ls)[9],
                                            const typename Store<S>::R (&ld)[9], const typename Store<S>::R (&F)[3],
                                            const typename Store<S>::R (&acc)[3],
                                            typename Store<S>::R* __restrict__ rs_next) {
    using R = typename Store<S>::R;
    using T = typename Store<S>::T;
    const size_t row = (size_t)g.nx * ((size_t)y + (size_t)g.ny * z);   // uniform
    const uint32_t xb = (uint32_t)x * (uint32_t)sizeof(R);
    const R Fx = F[0], Fy = F[1], Fz = F[2];
    R rho, ux, uy, uz;
    if constexpr (SGS) {
        R st[6];
        collide_lines<R, false, VAR, true, S == 3>(h, ls, ld, Fx, Fy, Fz, L.P, rho, ux, uy, uz, acc, st);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            __builtin_nontemporal_store(st[k], row_at<SB>(rs_next + (size_t)k * g.N + row, xb));
    } else {
        (void)acc; (void)rs_next;
        collide_lines<R, LES, VAR, false, S == 3>(h, ls, ld, Fx, Fy, Fz, L.P, rho, ux, uy, uz);
    }
    const uint32_t xt = (uint32_t)x * (uint32_t)sizeof(T);
#pragma unroll
    for (int i = 0; i < 27; ++i)
        __builtin_nontemporal_store(to_store<S>(h[i], i, L.P.rho0), row_at<SB>(dst + row_base(g, i, y, z), xt));
}

// SGS: the sub-grid stress acts as a force (rs_prev read, rs_next written).
// XL: one workgroup covers each grid row (nx <= blockDim.x, no walls in the
// launch), so the x-shifted values go through LDS (gather_xlds); otherwise
// each lane loads its shifted values itself (gather), looping over x when the
// grid has one workgroup per row (g.rowloop).
// FP16 storage is bound by instruction issue: five waves per SIMD (at most 96
// vector registers, which it fits without spilling) measured 3 % faster; the
// other modes gained nothing or spilled.
template <int S, bool WALLS, bool LES, bool FFIELD, bool VAR, bool SGS = false, bool XL = true>
__global__ void __launch_bounds__(256, (S == 3 && !SGS) ? 5 : 1) k_step(const typename Store<S>::T* __restrict__ src,
                                              typename Store<S>::T* __restrict__ dst,
                                              const typename Store<S>::R* __restrict__ force, const Geom g,
                                              const Launch<typename Store<S>::R> L,
                                              const typename Store<S>::R* __restrict__ rs_prev = nullptr,
                                              typename Store<S>::R* __restrict__ rs_next = nullptr) {
    using R = typename Store<S>::R;
    // Scalar-base addressing (at_row) for FP16 storage, which is bound by
    // instruction issue: 63 fewer vector instructions per wave, 4.8 % faster at
    // 512^3. The memory-bound modes measured 0.4-2 % slower with it (the extra
    // scalar work) and keep the vector addresses.
    constexpr bool SB = S == 3;
    int bx, y, z;
    block_coords(g.xcd, bx, y, z);
    y = g.ybase + y * g.ystride;
    z += g.zbase;
    if constexpr (XL) {
        static_assert(!WALLS, "the LDS gather is for periodic rows");
        const int x = threadIdx.x;
        const bool act = x < g.nx;
        // the stress and force loads go out with the population loads, in the
        // same memory round trip
        R sv[SGS ? 18 : 1], F[3];
        if constexpr (SGS) sgs_load<R, SB>(rs_prev, g, act ? x : 0, y, z, sv);
        row_force<R, FFIELD, SB>(force, g, L, act ? x : 0, y, z, F);
        typename Store<S>::T t[27];
        gather_xlds<S, SB>(src, g, x, act, y, z, t, [&]() {
            if constexpr (FFIELD) {
#pragma unroll
                for (int d = 0; d < 3; ++d) asm volatile("" : "+v"(F[d]));
            }
            if constexpr (SGS) {
#pragma unroll
                for (int k = 0; k < 18; ++k) asm volatile("" : "+v"(sv[k]));
            }
        });
        R h[27], ls[9], ld[9];
        if constexpr (S == 3) {
            // the z-line sums straight from the FP16 values (no conversions)
#pragma unroll
            for (int l = 0; l < 9; ++l)
                mix_line<0>(__builtin_bit_cast(uint16_t, t[l]), __builtin_bit_cast(uint16_t, t[l + 9]),
                            __builtin_bit_cast(uint16_t, t[l + 18]), ls[l], ld[l], h[l]);
        } else {
#pragma unroll
            for (int i = 0; i < 27; ++i) h[i] = from_store<S>(t[i], i, L.P.rho0);
            zline_sums(h, ls, ld);
        }
        R acc[3];
        if constexpr (SGS) sgs_combine(sv, acc);
        if (act) finish_cell<S, LES, VAR, SGS, SB>(dst, g, L, x, y, z, h, ls, ld, F, acc, rs_next);
    } else {
        if constexpr (SB) {
            if (!g.rowloop) {   // one cell per lane, no loop around the accesses
                const int x = bx * blockDim.x + threadIdx.x;
                if (x < g.nx) {
                    R acc[3], F[3];
                    if constexpr (SGS) sgs_accel<R, true>(rs_prev, g, x, y, z, acc);
                    R h[27], ls[9], ld[9];
                    gather<S, WALLS, 0, false, true>(src, g, x, y, z, L, h);
                    row_force<R, FFIELD, true>(force, g, L, x, y, z, F);
                    zline_sums(h, ls, ld);
                    finish_cell<S, LES, VAR, SGS, true>(dst, g, L, x, y, z, h, ls, ld, F, acc, rs_next);
                }
                return;
            }
        }
        for (int x = bx * blockDim.x + threadIdx.x; x < g.nx; x += gridDim.x * blockDim.x) {
            R acc[3], F[3];
            if constexpr (SGS) sgs_accel(rs_prev, g, x, y, z, acc);
            R h[27], ls[9], ld[9];
            gather<S, WALLS, 0, false>(src, g, x, y, z, L, h);
            row_force<R, FFIELD>(force, g, L, x, y, z, F);
            zline_sums(h, ls, ld);
            finish_cell<S, LES, VAR, SGS>(dst, g, L, x, y, z, h, ls, ld, F, acc, rs_next);
        }
    }
}

// ---------------------------------------------------------------- FP16 step, two cells per lane
// Non-temporal store of a 32-bit pair at a workgroup-uniform row pointer plus a
// lane offset. (Written out as an inline-assembly store with a scalar base it
// measured 0.7 % faster, but the compiler's hazard handling does not see the
// scalar base register of an assembly statement: the five wait states a
// memory instruction needs after v_readfirstlane writes its base register are
// then missing, and a store may use a stale address. Kept as compiler code.)
__device__ __forceinline__ void store_pair(uint32_t* row, uint32_t lane_bytes, uint32_t v) {
    __builtin_nontemporal_store(v, at_row(row, lane_bytes));
}

// FP16-shifted storage is bound by instruction issue rather than by HBM: the
// loads, stores, conversions and addresses are a large part of its work. Here
// each lane takes the two adjacent cells x = 2t and 2t + 1 of a periodic row
// (nx even, nx <= 2 blockDim.x, one workgroup per row): every population row is
// read and written as aligned 32-bit pairs, half the memory instructions of one
// cell per lane. Of the 18 rows with e_x != 0 each pair needs one value from
// the neighbouring pair (x - 1 for e_x = +1, x + 2 for e_x = -1), exchanged
// through LDS as in gather_xlds. The two cells then collide one after the
// other with the same arithmetic as k_step, so the results are bitwise those of
// the one-cell kernels.
template <bool LES, bool FFIELD, bool VAR>
__global__ void __launch_bounds__(256) k_step_f16pair(const _Float16* __restrict__ src, _Float16* __restrict__ dst,
                                                      const float* __restrict__ force, const Geom g,
                                                      const Launch<float> L) {
    using T = _Float16;
    __shared__ uint16_t sm[18][256];
    int bx, y, z;
    block_coords(g.xcd, bx, y, z);
    y = g.ybase + y * g.ystride;
    z += g.zbase;
    const int t = threadIdx.x;
    const int np = g.nx >> 1;   // pairs in the row
    const bool act = t < np;
    const int tp = act ? t : 0;   // idle lanes read pair 0 and fill LDS columns nobody reads
    const int ys[3] = {y == g.ny - 1 ? 0 : y + 1, y, y == 0 ? g.ny - 1 : y - 1};
    const int zs[3] = {z == g.nz - 1 ? 0 : z + 1, z, z == 0 ? g.nz - 1 : z - 1};
    const uint32_t rb = (uint32_t)g.nx * (uint32_t)sizeof(T);
    const uint32_t xt = (uint32_t)tp * 4u;
    uint32_t raw[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int ix = i % 3, iy = (i / 3) % 3, iz = i / 9;
        const T* grp = src + row_base(g, i - ix, ys[iy], zs[iz]);
        // non-temporal: every pair is read once per step (measured 3.5 % faster at 512^3)
        raw[i] = __builtin_nontemporal_load(at_row((const uint32_t*)grp, xt + (uint32_t)ix * rb));
    }
    float F[2][3];
    if constexpr (FFIELD) {
        const size_t row = (size_t)g.nx * ((size_t)y + (size_t)g.ny * z);   // uniform
        const uint32_t xb = (uint32_t)tp * 8u;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float2_t v = *at_row((const float2_t*)(force + (size_t)d * g.N + row), xb);
            F[0][d] = v.x;
            F[1][d] = v.y;
        }
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) F[0][d] = F[1][d] = L.F[d];
    }
    // e_x = -1 (ix = 0, source x + 1): the pair to the left needs this pair's
    // low value; e_x = +1 (ix = 2, source x - 1): the pair to the right needs
    // the high value
#pragma unroll
    for (int i = 0; i < 27; ++i)
        if (i % 3 != 1) sm[(i / 3) * 2 + (i % 3) / 2][t] = (uint16_t)(i % 3 == 0 ? raw[i] & 0xffffu : raw[i] >> 16);
#pragma unroll
    for (int i = 1; i < 27; i += 3) asm volatile("" : "+v"(raw[i]));
    if constexpr (FFIELD) {
#pragma unroll
        for (int d = 0; d < 3; ++d) asm volatile("" : "+v"(F[0][d]), "+v"(F[1][d]));
    }
    __syncthreads();
    const int tn = tp + 1 == np ? 0 : tp + 1, tv = tp == 0 ? np - 1 : tp - 1;
    float rho, ux, uy, uz;
    // cell x = 2t: e_x = 0 from the low halves, e_x = -1 from the high halves,
    // e_x = +1 the left pair's high values (LDS)
    float h[27], ls[9], ld[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
        const int ix = l % 3;
        if (ix == 1) mix_line<0>(raw[l], raw[l + 9], raw[l + 18], ls[l], ld[l], h[l]);
        else if (ix == 0) mix_line<1>(raw[l], raw[l + 9], raw[l + 18], ls[l], ld[l], h[l]);
        else {
            const int k = (l / 3) * 2 + 1;   // LDS row of population i = l + 9 iz: (i / 3) * 2 + 1
            mix_line<0>(sm[k][tv], sm[k + 6][tv], sm[k + 12][tv], ls[l], ld[l], h[l]);
        }
    }
    collide_lines<float, LES, VAR, false, true>(h, ls, ld, F[0][0], F[0][1], F[0][2], L.P, rho, ux, uy, uz);
    // cell x = 2t + 1: e_x = 0 from the high halves, e_x = +1 from the low
    // halves, e_x = -1 the right pair's low values (LDS)
    float h2[27];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
        const int ix = l % 3;
        if (ix == 1) mix_line<1>(raw[l], raw[l + 9], raw[l + 18], ls[l], ld[l], h2[l]);
        else if (ix == 2) mix_line<0>(raw[l], raw[l + 9], raw[l + 18], ls[l], ld[l], h2[l]);
        else {
            const int k = (l / 3) * 2;
            mix_line<0>(sm[k][tn], sm[k + 6][tn], sm[k + 12][tn], ls[l], ld[l], h2[l]);
        }
    }
    collide_lines<float, LES, VAR, false, true>(h2, ls, ld, F[1][0], F[1][1], F[1][2], L.P, rho, ux, uy, uz);
    if (act) {
#pragma unroll
        for (int i = 0; i < 27; ++i) store_pair((uint32_t*)(dst + row_base(g, i, y, z)), xt, pack_f16(h[i], h2[i]));
    }
}

// ---------------------------------------------------------------- in-place streaming
// One buffer, two kinds of step (the AA pattern of Bailey et al. 2009):
//   even: read fbar_i(x) from plane i of x, collide, write fbar~_i(x) to plane
//         26 - i of x (every access is to the thread's own cell);
//   odd:  read fbar_i(x) from plane 26 - i of x - e_i (gather MODE 2), collide,
//         write fbar~_i(x) to plane i of x + e_i, or, towards a wall, to plane
//         26 - i of x itself (the next even read adds the wall term);
// after an odd step the buffer is back in the natural arrangement. Each
// location is read and written by the same thread within a step, so the
// update is race-free in place. The collision and its arithmetic are those of
// the two-buffer step, so results are bitwise identical.
template <int S, bool WALLS, bool LES, bool FFIELD, bool VAR, bool ODD>
__global__ void __launch_bounds__(256) k_step_inplace(typename Store<S>::T* buf,
                                                      const typename Store<S>::R* __restrict__ force, const Geom g,
                                                      const Launch<typename Store<S>::R> L) {
    using R = typename Store<S>::R;
    using T = typename Store<S>::T;
    int bx, y, z;
    block_coords(g.xcd, bx, y, z);
    y = g.ybase + y * g.ystride;
    z += g.zbase;
    for (int x = bx * blockDim.x + threadIdx.x; x < g.nx; x += gridDim.x * blockDim.x) {
        R h[27];
        if constexpr (ODD) gather<S, WALLS, 2>(buf, g, x, y, z, L, h);
        else gather<S, WALLS, 1>(buf, g, x, y, z, L, h);
        const size_t row = (size_t)g.nx * ((size_t)y + (size_t)g.ny * z);
        R Fx, Fy, Fz;
        if constexpr (FFIELD) {
            Fx = force[row + x];
            Fy = force[(size_t)g.N + row + x];
            Fz = force[2 * (size_t)g.N + row + x];
        } else {
            Fx = L.F[0];
            Fy = L.F[1];
            Fz = L.F[2];
        }
        R rho, ux, uy, uz;
        collide<R, LES, VAR, false, S == 3>(h, Fx, Fy, Fz, L.P, rho, ux, uy, uz);
        if constexpr (!ODD) {
            const uint32_t xt = (uint32_t)x * (uint32_t)sizeof(T);
#pragma unroll
            for (int i = 0; i < 27; ++i)
                __builtin_nontemporal_store(to_store<S>(h[i], 26 - i, L.P.rho0),
                                            (T*)((char*)(buf + row_base(g, 26 - i, y, z)) + xt));
        } else {
            const int xs[3] = {x == 0 ? g.nx - 1 : x - 1, x, x == g.nx - 1 ? 0 : x + 1};   // x + ex
            const int ys[3] = {y == 0 ? g.ny - 1 : y - 1, y, y == g.ny - 1 ? 0 : y + 1};
            const int zs[3] = {z == 0 ? g.nz - 1 : z - 1, z, z == g.nz - 1 ? 0 : z + 1};
            // one uniform pointer per target row (ey, ez), the row-in-group offset
            // folded into the per-lane offsets (as in the gather)
            uint32_t vo[3];
#pragma unroll
            for (int ix = 0; ix < 3; ++ix) vo[ix] = ((uint32_t)xs[ix] + (uint32_t)ix * (uint32_t)g.nx) * (uint32_t)sizeof(T);
#pragma unroll
            for (int i = 0; i < 27; ++i) {
                const int ix = i % 3, iy = (i / 3) % 3, iz = i / 9;
                if constexpr (WALLS) {
                    const bool to_lo = (iy == 0) && (y == 0);
                    const bool to_hi = (iy == 2) && (y == g.ny - 1);
                    if (to_lo || to_hi) {
                        const int o = 26 - i;
                        __builtin_nontemporal_store(to_store<S>(h[i], o, L.P.rho0), buf + row_base(g, o, y, z) + x);
                        continue;
                    }
                }
                __builtin_nontemporal_store(to_store<S>(h[i], i, L.P.rho0),
                                            (T*)((char*)(buf + row_base(g, i - ix, ys[iy], zs[iz])) + vo[ix]));
            }
        }
    }
}

// ---------------------------------------------------------------- scatter of canonical populations
// Writes canonical fbar(n) at cell (x,y,z) into the internal (pull) layout:
// population i goes to the upstream cell x - e_i, or, when that is a wall, to
// the opposite plane of the same cell minus the wall term.
template <int S, bool WALLS, typename R = typename Store<S>::R>
__device__ __forceinline__ void scatter(typename Store<S>::T* __restrict__ dst, const Geom g, int x, int y, int z,
                                        const Launch<R>& L, const R (&h)[27]) {
    if (g.aa) {   // in-place streaming: a state is set in the natural (even) arrangement,
                  // populations from a wall without their wall term
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            R v = h[i];
            if constexpr (WALLS) {
                const int iy = (i / 3) % 3;
                const bool from_lo = (iy == 2) && (y == 0);
                const bool from_hi = (iy == 0) && (y == g.ny - 1);
                if (from_lo || from_hi) v = sub_rn(v, from_lo ? L.wt_lo[i] : L.wt_hi[i]);
            }
            dst[row_base(g, i, y, z) + x] = to_store<S>(v, i, L.P.rho0);
        }
        return;
    }
    const int xs[3] = {x == g.nx - 1 ? 0 : x + 1, x, x == 0 ? g.nx - 1 : x - 1};
    const int ys[3] = {y == g.ny - 1 ? 0 : y + 1, y, y == 0 ? g.ny - 1 : y - 1};
    const int zs[3] = {z == g.nz - 1 ? 0 : z + 1, z, z == 0 ? g.nz - 1 : z - 1};
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int ix = i % 3, iy = (i / 3) % 3, iz = i / 9;
        if constexpr (WALLS) {
            const bool from_lo = (iy == 2) && (y == 0);
            const bool from_hi = (iy == 0) && (y == g.ny - 1);
            if (from_lo || from_hi) {
                const int o = 26 - i;
                const R v = sub_rn(h[i], from_lo ? L.wt_lo[i] : L.wt_hi[i]);
                dst[row_base(g, o, y, z) + x] = to_store<S>(v, o, L.P.rho0);
                continue;
            }
        }
        dst[row_base(g, i, ys[iy], zs[iz]) + xs[ix]] = to_store<S>(h[i], i, L.P.rho0);
    }
}

template <int S, bool WALLS, bool FFIELD>
__global__ void __launch_bounds__(256) k_init_equilibrium(typename Store<S>::T* __restrict__ dst,
                                                          const typename Store<S>::R* __restrict__ force,
                                                          const void* __restrict__ rho_in, const void* __restrict__ u_in,
                                                          int dt, const Geom g, const Launch<typename Store<S>::R> L) {
    using R = typename Store<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const int c = x + g.nx * (y + g.ny * z);
    const R rho = rho_in ? static_cast<R>(as_double(rho_in, dt, c)) : L.P.rho0;
    const R ux = static_cast<R>(as_double(u_in, dt, c));
    const R uy = static_cast<R>(as_double(u_in, dt, (size_t)g.N + c));
    const R uz = static_cast<R>(as_double(u_in, dt, 2 * (size_t)g.N + c));
    R Fx, Fy, Fz;
    cell_force<R, FFIELD>(force, g, c, L, Fx, Fy, Fz);
    R h[27];
    equilibrium(h, rho, ux, uy, uz, Fx, Fy, Fz, L.P.rho0, L.P.rc != 0);
    scatter<S, WALLS>(dst, g, x, y, z, L, h);
}

template <int S, bool WALLS>
__global__ void __launch_bounds__(256) k_set_populations(typename Store<S>::T* __restrict__ dst,
                                                         const void* __restrict__ f, int dt, const Geom g,
                                                         const Launch<typename Store<S>::R> L) {
    using R = typename Store<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const int c = x + g.nx * (y + g.ny * z);
    R h[27];
#pragma unroll
    for (int i = 0; i < 27; ++i)
        h[i] = static_cast<R>(as_double(f, dt, (size_t)i * g.N + c) - (double)L.P.rho0 * (double)w27<double>(i));
    scatter<S, WALLS>(dst, g, x, y, z, L, h);
}

// ---------------------------------------------------------------- read-out
// mode 0: canonical populations into out0 (27 planes); mode 1: rho into out0
// (1 plane) and u into out1 (3 planes)
template <int S, bool WALLS, bool FFIELD>
__global__ void __launch_bounds__(256) k_read(const typename Store<S>::T* __restrict__ src,
                                              const typename Store<S>::R* __restrict__ force, void* __restrict__ out0,
                                              void* __restrict__ out1, int dt, int mode, const Geom g,
                                              const Launch<typename Store<S>::R> L) {
    using R = typename Store<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const int c = x + g.nx * (y + g.ny * z);
    R h[27];
    gather_any<S, WALLS>(src, g, x, y, z, L, h);
    auto put = [&](void* out, size_t k, double v) {
        if (dt == 0) static_cast<double*>(out)[k] = v;
        else static_cast<float*>(out)[k] = static_cast<float>(v);
    };
    if (mode == 0) {
#pragma unroll
        for (int i = 0; i < 27; ++i)
            put(out0, (size_t)i * g.N + c, (double)h[i] + (double)L.P.rho0 * w27<double>(i));
        return;
    }
    R Fx, Fy, Fz;
    cell_force<R, FFIELD>(force, g, c, L, Fx, Fy, Fz);
    R drho, jx, jy, jz;
    mass_momentum(h, drho, jx, jy, jz);
    const R rho = L.P.rho0 + drho;
    if (L.rs_prev) {   // sub-grid stress as a force: F + rho a'
        R a[3];
        sgs_accel(L.rs_prev, g, x, y, z, a);
        Fx += rho * a[0];
        Fy += rho * a[1];
        Fz += rho * a[2];
    }
    const R rho_u = L.P.rc ? L.P.rho0 : rho;   // reduced compressibility: rho0 u = j + F/2
    put(out0, c, (double)rho);
    put(out1, c, (double)((jx + R(0.5) * Fx) / rho_u));
    put(out1, (size_t)g.N + c, (double)((jy + R(0.5) * Fy) / rho_u));
    put(out1, 2 * (size_t)g.N + c, (double)((jz + R(0.5) * Fz) / rho_u));
}

// ---------------------------------------------------------------- adjoint
// Discrete adjoint of one step. The forward step maps fbar(n) -> fbar(n+1)
// by collision C (per cell) and streaming P: fbar_i(x, n+1) = fbar~_i(x - e_i, n).
// Its transpose gathers lam~_i(x) = lam_i(x + e_i, n+1); then
// lam(x, n) = J_C(x)^T lam~(x) and grad_F(x) += (dC/dF)^T lam~(x). lambda is
// held in the populations' row layout, element (i, x, y, z) at
// ((z ny + y) 27 + i) nx + x, so that its gather reads three adjacent rows in
// each of nine row groups, as the state's does (measured against 27 separate
// planes: 133.7 -> 123.0 us at 128^3, 1034 -> 1026 us at 256^3). WALLS: a
// post-collision population that leaves towards a wall comes back as the
// opposite population of its own cell (plus a constant), so there
// lam~_i(x) = lam_{26-i}(x, n+1). LES: the collision with the eddy rate;
// VAR: with the Sec. 12-13 operators (L.P.rc, L.P.fact).
template <int S, bool FFIELD, bool WALLS, bool LES, bool VAR>
__global__ void __launch_bounds__(256) k_adjoint(const typename Store<S>::T* __restrict__ state,
                                                 const typename Store<S>::R* __restrict__ lam_in,
                                                 typename Store<S>::R* __restrict__ lam_out,
                                                 typename Store<S>::R* __restrict__ grad_F,
                                                 const typename Store<S>::R* __restrict__ force, const Geom g,
                                                 const Launch<typename Store<S>::R> L) {
    using R = typename Store<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z + g.zbase;
    if (x >= g.nx) return;
    // fbar(n): ordinary loads also for the x-shifted rows, so that the cache
    // lines a wave shares with its neighbour stay in L2 for the second reader
    // (with non-temporal loads they were fetched from HBM again: 256 against
    // 240 B/cell of reads, 3 % slower at 256^3)
    R h[27];
    gather<S, WALLS, 0, false>(state, g, x, y, z, L, h);
    // lambda at x + e_i: the rows (y + ey, z + ez) are block-uniform (scalar
    // registers); only the x offset (x - 1, x, x + 1 with wrap) is per lane.
    // (An LDS exchange of the x-shifted values, as in the step kernel, was
    // measured slower here: it costs this kernel its occupancy.)
    const size_t N = (size_t)g.N, nx = (size_t)g.nx;
    const uint32_t xo[3] = {(uint32_t)(x == 0 ? g.nx - 1 : x - 1) * (uint32_t)sizeof(R), (uint32_t)x * (uint32_t)sizeof(R),
                            (uint32_t)(x == g.nx - 1 ? 0 : x + 1) * (uint32_t)sizeof(R)};
    const int yd[3] = {y == 0 ? g.ny - 1 : y - 1, y, y == g.ny - 1 ? 0 : y + 1};
    const int zd[3] = {z == 0 ? g.nz - 1 : z - 1, z, z == g.nz - 1 ? 0 : z + 1};
    R lam[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        if constexpr (WALLS) {
            const int iy = (i / 3) % 3;   // e_y = iy - 1
            if ((iy == 0 && y == 0) || (iy == 2 && y == g.ny - 1)) {
                const R* own = lam_in + nx * (((size_t)y + (size_t)g.ny * z) * 27 + (size_t)(26 - i));
                lam[i] = __builtin_nontemporal_load((const R*)((const char*)own + xo[1]));
                continue;
            }
        }
        // as for the state: the rows read at x are read once (non-temporal),
        // the x-shifted ones keep ordinary loads so that the lines a wave
        // shares with its neighbour stay in L2 (non-temporal loads of the
        // aligned rows: 1,015 -> 1,000 us at 256^3, 124.7 -> 115.8 us at 128^3)
        const R* rowp = lam_in + nx * (((size_t)yd[(i / 3) % 3] + (size_t)g.ny * zd[i / 9]) * 27 + (size_t)i);
        if (i % 3 == 1) lam[i] = __builtin_nontemporal_load((const R*)((const char*)rowp + xo[1]));
        else lam[i] = *(const R*)((const char*)rowp + xo[i % 3]);
    }
    const size_t row = nx * ((size_t)y + (size_t)g.ny * z);
    R F[3], g0[3];
    row_force<R, FFIELD>(force, g, L, x, y, z, F);
    // the force gradient so far, read with the other inputs rather than at the end
#pragma unroll
    for (int d = 0; d < 3; ++d) g0[d] = grad_F[(size_t)d * N + row + x];
    R gF[3] = {R(0), R(0), R(0)};
    collide_adjoint<R, LES, VAR>(h, lam, F[0], F[1], F[2], L.P, gF);
#pragma unroll
    for (int i = 0; i < 27; ++i) __builtin_nontemporal_store(lam[i], lam_out + (row * 27 + (size_t)i * nx) + x);
#pragma unroll
    for (int d = 0; d < 3; ++d) grad_F[(size_t)d * N + row + x] = g0[d] + gF[d];
}

// Seeds of E = sum rho |u|^2 / 2: dE/dfbar_i = u.e_i - |u|^2/2 (in the row
// layout of lambda), dE/dF = u/2. With reduced compressibility (rho0 u =
// sum fbar e + F/2, Sec. 12): dE/dfbar_i = (rho/rho0) u.e_i + |u|^2/2,
// dE/dF = (rho/rho0) u/2.
template <int S, bool FFIELD, bool WALLS = false>
__global__ void __launch_bounds__(256) k_energy_seed(const typename Store<S>::T* __restrict__ state,
                                                     typename Store<S>::R* __restrict__ lam_out,
                                                     typename Store<S>::R* __restrict__ grad_F,
                                                     const typename Store<S>::R* __restrict__ force, const Geom g,
                                                     const Launch<typename Store<S>::R> L) {
    using R = typename Store<S>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const int c = x + g.nx * (y + g.ny * z);
    R h[27];
    gather<S, WALLS>(state, g, x, y, z, L, h);
    R Fx, Fy, Fz;
    cell_force<R, FFIELD>(force, g, c, L, Fx, Fy, Fz);
    R drho, jx, jy, jz;
    mass_momentum(h, drho, jx, jy, jz);
    const bool rc = L.P.rc != 0;
    const R rho = L.P.rho0 + drho;
    const R inv_rho_u = rc ? R(1) / L.P.rho0 : R(1) / rho;
    const R ux = (jx + R(0.5) * Fx) * inv_rho_u, uy = (jy + R(0.5) * Fy) * inv_rho_u, uz = (jz + R(0.5) * Fz) * inv_rho_u;
    const R hu2 = R(0.5) * (ux * ux + uy * uy + uz * uz);
    const R s = rc ? rho * inv_rho_u : R(1);   // rho / rho0, or 1
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int ex = i % 3 - 1, ey = (i / 3) % 3 - 1, ez = i / 9 - 1;
        lam_out[((size_t)(y + g.ny * z) * 27 + (size_t)i) * (size_t)g.nx + x] =
            s * (R(ex) * ux + R(ey) * uy + R(ez) * uz) + (rc ? hu2 : -hu2);
    }
    grad_F[c] = R(0.5) * s * ux;
    grad_F[(size_t)g.N + c] = R(0.5) * s * uy;
    grad_F[2 * (size_t)g.N + c] = R(0.5) * s * uz;
}

// ---------------------------------------------------------------- FP64 reductions
// Partial sums per workgroup. The lattice is cut into tiles of one workgroup
// width along a grid row, numbered x chunk fastest, then y, then z; workgroup b
// (linear index over the launch grid) combines, lane by lane, the cells of
// tiles b, b + B, b + 2B, ... (B workgroups in the launch) in that order, then
// reduces over its lanes in a fixed tree. Launched with one workgroup per tile
// it visits exactly its own tile; launched with fewer workgroups the partials
// need only 8 B doubles, whatever the lattice size.
template <int S, bool WALLS, bool FFIELD>
__global__ void __launch_bounds__(256) k_reduce_partial(const typename Store<S>::T* __restrict__ src,
                                                        const typename Store<S>::R* __restrict__ force,
                                                        double* __restrict__ partial, const Geom g,
                                                        const Launch<typename Store<S>::R> L) {
    using R = typename Store<S>::R;
    const uint32_t gx = (uint32_t)((g.nx + (int)blockDim.x - 1) / (int)blockDim.x);
    const uint64_t ntiles = (uint64_t)gx * (uint64_t)g.ny * (uint64_t)g.nz;
    const uint64_t nblocks = (uint64_t)gridDim.x * gridDim.y * gridDim.z;
    const uint64_t b = blockIdx.x + (uint64_t)gridDim.x * (blockIdx.y + (uint64_t)gridDim.y * blockIdx.z);
    double v[8] = {0, 0, 0, 0, 0, 0, 1.0e300, 0};
    for (uint64_t t = b; t < ntiles; t += nblocks) {
        const int x = (int)(t % gx) * (int)blockDim.x + (int)threadIdx.x;
        const uint64_t r = t / gx;
        const int y = (int)(r % (uint64_t)g.ny), z = (int)(r / (uint64_t)g.ny);
        if (x >= g.nx) continue;
        const int c = x + g.nx * (y + g.ny * z);
        R h[27];
        gather_any<S, WALLS>(src, g, x, y, z, L, h);
        double hd[27];
#pragma unroll
        for (int i = 0; i < 27; ++i) hd[i] = (double)h[i];
        double drho, jx, jy, jz;
        mass_momentum(hd, drho, jx, jy, jz);
        R Fx, Fy, Fz;
        cell_force<R, FFIELD>(force, g, c, L, Fx, Fy, Fz);
        if (L.rs_prev) {   // sub-grid stress as a force: F + rho a' (rho in the compute type)
            R a[3];
            sgs_accel(L.rs_prev, g, x, y, z, a);
            const R rho_r = L.P.rho0 + (R)drho;
            Fx += rho_r * a[0];
            Fy += rho_r * a[1];
            Fz += rho_r * a[2];
        }
        const double rho = (double)L.P.rho0 + drho;
        const double rho_u = L.P.rc ? (double)L.P.rho0 : rho;
        const double ux = (jx + 0.5 * (double)Fx) / rho_u, uy = (jy + 0.5 * (double)Fy) / rho_u,
                     uz = (jz + 0.5 * (double)Fz) / rho_u;
        const double px = rho * ux, py = rho * uy, pz = rho * uz;
        const double u2 = ux * ux + uy * uy + uz * uz;
        const bool bad = !isfinite(rho) || !isfinite(u2);
        double w[8];
        w[0] = rho;
        w[1] = px;
        w[2] = py;
        w[3] = pz;
        w[4] = 0.5 * rho * u2;
        w[5] = bad ? 1.0 : 0.0;
        w[6] = bad ? 1.0e300 : rho;
        w[7] = bad ? 0.0 : sqrt(u2);
        if (bad) { w[0] = w[1] = w[2] = w[3] = w[4] = 0.0; }
        combine(v, w);
    }
    block_reduce(v, partial + 8 * b);
}

__global__ void __launch_bounds__(256) k_reduce_final(const double* __restrict__ partial, size_t nparts,
                                                      double* __restrict__ out) {
    double v[8] = {0, 0, 0, 0, 0, 0, 1.0e300, 0};
    for (size_t b = threadIdx.x; b < nparts; b += blockDim.x) {
        double w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) w[k] = partial[8 * b + k];
        combine(v, w);
    }
    block_reduce(v, out);
}

// ---------------------------------------------------------------- plain copy
// Reference streaming kernel used to calibrate bandwidth and hardware byte
// counters against a known size: one 16-byte vector per thread, non-temporal
// load and store, 64-thread workgroups (the fastest plain copy form measured
// on MI355X, 4 GiB each way, on two machines: 6.67 and 6.73 TB/s, against 6.52
// and 6.49 with 256-thread workgroups, 6.35 with 512, 6.18 with 1024, 6.21-6.26
// with an ordinary load; two or more vectors per thread and grid-stride loops
// were slower still, 4.1-6.1 TB/s).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_zero(unsigned int* __restrict__ dst, size_t n) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = 0u;
}
__global__ void __launch_bounds__(256) k_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst, size_t n16) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + k), dst + k);
}

// ---------------------------------------------------------------- launch helpers
// Rows of up to 256 cells get one workgroup of the next width in {64, 128,
// 256} (so that the LDS gather applies); wider rows workgroups of 256.
static dim3 grid_for_step(const Geom& g, int& bx) {
    bx = g.nx <= 64 ? 64 : (g.nx <= 128 ? 128 : 256);
    return dim3(g.rowloop ? 1 : (g.nx + bx - 1) / bx, g.yrows, g.nz);
}

// With walls, only the rows y = 0 and y = ny - 1 need the bounce-back code:
// the interior rows run the periodic kernel (its y +- 1 never wraps there) and
// the two wall rows a kernel of their own, so that the wall terms and extra
// row pointers do not burden the registers of every workgroup.
template <typename F>
static hipError_t split_wall_rows(const LaunchArgs& a, F&& launch) {
    if (!a.walls) return launch(a, false);
    const int ny = a.g.ny;
    if (ny > 2) {
        LaunchArgs in = a;
        in.g.ybase = 1;
        in.g.ystride = 1;
        in.g.yrows = ny - 2;
        hipError_t e = launch(in, false);
        if (e != hipSuccess) return e;
    }
    LaunchArgs wl = a;
    wl.g.ybase = 0;
    wl.g.ystride = ny > 1 ? ny - 1 : 1;
    wl.g.yrows = ny > 1 ? 2 : 1;
    return launch(wl, true);
}

static dim3 grid_for(const Geom& g, int& bx) {
    bx = g.nx >= 256 ? 256 : (g.nx >= 128 ? 128 : 64);
    return dim3((g.nx + bx - 1) / bx, g.ny, g.nz);
}

template <typename R>
static Launch<R> make_launch(const LaunchArgs& a) {
    Launch<R> L;
    L.P.rho0 = (R)a.rho0;
    L.P.ws = (R)a.omega_shear;
    L.P.wb = (R)a.omega_bulk;
    L.P.w3a = (R)a.omega3[0];
    L.P.w3b = (R)a.omega3[1];
    L.P.w3c = (R)a.omega3[2];
    L.P.w4a = (R)a.omega4[0];
    L.P.w4b = (R)a.omega4[1];
    L.P.w5 = (R)a.omega5;
    L.P.w6 = (R)a.omega6;
    L.P.tau0 = (R)(1.0 / a.omega_shear);
    L.P.smag = (R)(18.0 * a.cs_smag * a.cs_smag);
    L.P.fact = (a.flags & 1u) ? 1 : 0;
    L.P.rc = (a.flags & 2u) ? 1 : 0;
    L.P.sgs = (a.flags & 4u) ? (R)(4.5 * a.cs_smag * a.cs_smag * a.omega_shear * a.omega_shear) : R(0);
    derive_coefficients(L.P);
    L.rs_prev = (a.flags & 4u) ? (const R*)a.stress_prev : nullptr;
    for (int d = 0; d < 3; ++d) L.F[d] = (R)a.force[d];
    for (int i = 0; i < 27; ++i) {
        const int e[3] = {i % 3 - 1, (i / 3) % 3 - 1, i / 9 - 1};
        const double w = (i % 3 == 1 ? 2.0 / 3.0 : 1.0 / 6.0) * ((i / 3) % 3 == 1 ? 2.0 / 3.0 : 1.0 / 6.0) *
                         (i / 9 == 1 ? 2.0 / 3.0 : 1.0 / 6.0);
        double dlo = 0.0, dhi = 0.0;
        for (int d = 0; d < 3; ++d) {
            dlo += e[d] * a.wall_u_lo[d];
            dhi += e[d] * a.wall_u_hi[d];
        }
        L.wt_lo[i] = (R)(6.0 * w * a.rho0 * dlo);
        L.wt_hi[i] = (R)(6.0 * w * a.rho0 * dhi);
    }
    return L;
}

// The LDS gather needs one workgroup per grid row (a single chunk of x) and
// periodic rows; the wall rows and wider rows take the per-lane gather, and so
// does every row when the caller asks for it (g.lanegather, a tuning hint).
static bool one_block_per_row(const Geom& g, const dim3& grid, int bx) { return grid.x == 1 && g.nx <= bx && !g.lanegather; }

// FP16 rows for the two-cells-per-lane kernel: an even number of 258 to 512
// cells (one workgroup of at most 256 lanes per row; rows of up to 256 cells
// take the one-cell LDS kernel, measured 3 % faster at 256^3), LDS exchange
// allowed, no row loop, and buffers aligned for 32-bit population pairs and
// 64-bit force pairs (every row then starts on such a boundary, as nx is even).
static bool pair_rows(const Geom& g, const void* src, const void* dst, const void* force) {
    const bool aligned = (uintptr_t)src % 4 == 0 && (uintptr_t)dst % 4 == 0 && (uintptr_t)force % 8 == 0;
    return aligned && g.nx % 2 == 0 && g.nx > 256 && g.nx <= 512 && !g.lanegather && !g.rowloop && !g.pairs_off;
}

// Occupancy caps by LDS reservation: with 60,000 bytes of the CU's 160 KB of
// LDS reserved per workgroup, at most two workgroups share a CU; with 40,960
// bytes, four (three for a kernel that holds 9 KB of its own). The reserved
// LDS itself is not used. Measured at 256^3 and 512^3, fewer resident rows per
// CU made the DRAM traffic of these kernels more efficient: the in-place pair
// of kernels with 4-byte populations on rows of at most 512 cells 3-6 % faster
// at two workgroups per CU (FP16: slower; rows of 1024 cells: not faster), the
// per-lane gather with 4-byte populations on rows of 257-512 cells 1-2 %
// faster at four, the two-cells-per-lane FP16 kernel about 1 % faster at
// three. The LDS-exchange step kernels are fastest at their full occupancy
// (six to seven workgroups).
constexpr unsigned kLdsTwoPerCu = 60000, kLdsFourPerCu = 40960, kLdsPairCap = 40960;

// A step over many z-planes runs as launches of at most kZChunk planes each:
// the end of each launch brings the eight XCDs back to the same planes, where
// over one long launch they drift apart and the planes being read and written
// at a time spread out. Measured (us per step, one launch / chunks of 128
// planes): 256^3 FP32 step (one workgroup per row) 591.6 / 578.2 and
// 596.0 / 586.5 on two machines, 256 x 256 x 1024 2,679 / 2,483; chunks of 64
// and 32 planes gained less or lost. The adjoint kernel gains as well (256^3
// FP32: 1,041 / 1,020 us; chunks of 64 the same there but 4 % slower at
// 128^3, chunks of 32 slower). Not faster, so kept in one launch: the
// FP16 two-cell kernel (2,665 / 2,701 us at 512^3), FP32-shifted rows of 512
// cells (5,192 / 5,208), FP64 rows of 512 cells (9,953 / 9,751 on one machine but
// 9,578 / 10,113 on another), the in-place kernels (256^3: 653 / 656 us), the
// wall rows and the D2Q9 step (8192^2: 869 us in one launch, 875-927 us in
// chunks of 4096-512 rows). The FP32 sub-grid-force step with one workgroup
// per row gains 1.1 % (769.4 / 761.2 us at 256^3).
constexpr int kZChunk = 128;
template <typename Launch1>
static hipError_t launch_z_chunks(const Geom& g, const dim3& grid, bool chunked, Launch1&& launch) {
    const int chunk = chunked && !g.one_launch && g.nz > kZChunk ? kZChunk : g.nz;
    for (int z0 = 0; z0 < g.nz; z0 += chunk) {
        Geom gg = g;
        gg.zbase = z0;
        launch(dim3(grid.x, grid.y, (unsigned)(g.nz - z0 < chunk ? g.nz - z0 : chunk)), gg);
        // the first failed launch ends the step (and is the error returned)
        if (const hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int S, bool W, bool LES, bool FF>
static hipError_t step_t(const LaunchArgs& a, const void* src, void* dst) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    const dim3 grid = grid_for_step(a.g, bx);
    const bool var = (a.flags & 3u) != 0;
    hipStream_t st = (hipStream_t)a.stream;
    const Launch<R> L = make_launch<R>(a);
    if constexpr (!W && S == 3) {
        if (pair_rows(a.g, src, dst, a.force_field)) {
            const dim3 gp(1, a.g.yrows, a.g.nz);
            const int bp = 256;   // one lane per pair of a row of 258-512 cells
            // with its own 9 KB of LDS, at most three workgroups per CU
            // (measured 0.8 and 1.3 % faster at 512^3 on two machines)
            if (var) k_step_f16pair<LES, FF, true><<<gp, bp, kLdsPairCap, st>>>((const T*)src, (T*)dst, (const R*)a.force_field, a.g, L);
            else k_step_f16pair<LES, FF, false><<<gp, bp, kLdsPairCap, st>>>((const T*)src, (T*)dst, (const R*)a.force_field, a.g, L);
            return hipGetLastError();
        }
    }
    if constexpr (!W) {
        if (one_block_per_row(a.g, grid, bx)) {
            return launch_z_chunks(a.g, grid, sizeof(T) == 4, [&](const dim3& gq, const Geom& gg) {
                if (var) k_step<S, W, LES, FF, true, false, true><<<gq, bx, 0, st>>>((const T*)src, (T*)dst, (const R*)a.force_field, gg, L);
                else k_step<S, W, LES, FF, false, false, true><<<gq, bx, 0, st>>>((const T*)src, (T*)dst, (const R*)a.force_field, gg, L);
            });
        }
    }
    const unsigned cap = sizeof(T) == 4 && a.g.nx > 256 && a.g.nx <= 512 ? kLdsFourPerCu : 0u;
    if (var) k_step<S, W, LES, FF, true, false, false><<<grid, bx, cap, st>>>((const T*)src, (T*)dst, (const R*)a.force_field, a.g, L);
    else k_step<S, W, LES, FF, false, false, false><<<grid, bx, cap, st>>>((const T*)src, (T*)dst, (const R*)a.force_field, a.g, L);
    return hipGetLastError();
}

template <int S, bool W, bool LES, bool FF>
static hipError_t step_inplace_t(const LaunchArgs& a, void* buf) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    const dim3 grid = grid_for_step(a.g, bx);
    const bool odd = a.g.aa == 2, var = (a.flags & 3u) != 0;
    hipStream_t st = (hipStream_t)a.stream;
    const Launch<R> L = make_launch<R>(a);
    const unsigned cap = sizeof(T) == 4 && a.g.nx <= 512 ? kLdsTwoPerCu : 0u;
    if (odd && var) k_step_inplace<S, W, LES, FF, true, true><<<grid, bx, cap, st>>>((T*)buf, (const R*)a.force_field, a.g, L);
    else if (odd) k_step_inplace<S, W, LES, FF, false, true><<<grid, bx, cap, st>>>((T*)buf, (const R*)a.force_field, a.g, L);
    else if (var) k_step_inplace<S, W, LES, FF, true, false><<<grid, bx, cap, st>>>((T*)buf, (const R*)a.force_field, a.g, L);
    else k_step_inplace<S, W, LES, FF, false, false><<<grid, bx, cap, st>>>((T*)buf, (const R*)a.force_field, a.g, L);
    return hipGetLastError();
}
template <int S, bool W>
static hipError_t step_inplace_w(const LaunchArgs& a, void* buf) {
    if (a.cs_smag > 0.0)
        return a.force_field ? step_inplace_t<S, W, true, true>(a, buf) : step_inplace_t<S, W, true, false>(a, buf);
    return a.force_field ? step_inplace_t<S, W, false, true>(a, buf) : step_inplace_t<S, W, false, false>(a, buf);
}
template <int S>
static hipError_t step_inplace_s(const LaunchArgs& a, void* buf) {
    if (a.g.aa != 1 && a.g.aa != 2) return hipErrorInvalidValue;
    return split_wall_rows(a, [&](const LaunchArgs& b, bool w) {
        return w ? step_inplace_w<S, true>(b, buf) : step_inplace_w<S, false>(b, buf);
    });
}

// Sub-grid stress as a force (periodic lattices, no eddy rate in the collision).
template <int S, bool FF>
static hipError_t step_sgs_t(const LaunchArgs& a, const void* src, void* dst) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    const dim3 grid = grid_for_step(a.g, bx);
    const bool var = (a.flags & 3u) != 0;
    const bool xl = one_block_per_row(a.g, grid, bx);
    hipStream_t st = (hipStream_t)a.stream;
    const Launch<R> L = make_launch<R>(a);
    const R* rp = (const R*)a.stress_prev;
    R* rn = (R*)a.stress_next;
    // the stress planes read by the y-neighbour rows favour the plain order
    // over runs of rows per XCD (measured 768 against 784 us at 256^3)
    Geom g = a.g;
    if (a.xcd_default && g.xcd >= 2) g.xcd = 0;
    // FP32 rows of one workgroup in chunks of planes, as the step without the
    // stress force (256^3: 769.4 -> 761.2 us)
    return launch_z_chunks(g, grid, sizeof(T) == 4 && xl, [&](const dim3& gq, const Geom& gg) {
        if (var && xl) k_step<S, false, false, FF, true, true, true><<<gq, bx, 0, st>>>((const T*)src, (T*)dst, (const R*)a.force_field, gg, L, rp, rn);
        else if (var) k_step<S, false, false, FF, true, true, false><<<gq, bx, 0, st>>>((const T*)src, (T*)dst, (const R*)a.force_field, gg, L, rp, rn);
        else if (xl) k_step<S, false, false, FF, false, true, true><<<gq, bx, 0, st>>>((const T*)src, (T*)dst, (const R*)a.force_field, gg, L, rp, rn);
        else k_step<S, false, false, FF, false, true, false><<<gq, bx, 0, st>>>((const T*)src, (T*)dst, (const R*)a.force_field, gg, L, rp, rn);
    });

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
    return split_wall_rows(a, [&](const LaunchArgs& b, bool w) {
        return w ? step_les<S, true>(b, src, dst) : step_les<S, false>(b, src, dst);
    });
}

template <int S, bool W, bool FF>
static hipError_t init_t(const LaunchArgs& a, void* dst, const void* rho, const void* u, int dt) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    const dim3 grid = grid_for(a.g, bx);
    k_init_equilibrium<S, W, FF><<<grid, bx, 0, (hipStream_t)a.stream>>>((T*)dst, (const R*)a.force_field, rho, u, dt,
                                                                         a.g, make_launch<R>(a));
    return hipGetLastError();
}

template <int S, bool W>
static hipError_t setpop_t(const LaunchArgs& a, void* dst, const void* f, int dt) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    const dim3 grid = grid_for(a.g, bx);
    k_set_populations<S, W><<<grid, bx, 0, (hipStream_t)a.stream>>>((T*)dst, f, dt, a.g, make_launch<R>(a));
    return hipGetLastError();
}

template <int S, bool W, bool FF>
static hipError_t read_t(const LaunchArgs& a, const void* src, void* out0, void* out1, int dt, int mode) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    const dim3 grid = grid_for(a.g, bx);
    k_read<S, W, FF><<<grid, bx, 0, (hipStream_t)a.stream>>>((const T*)src, (const R*)a.force_field, out0, out1, dt,
                                                            mode, a.g, make_launch<R>(a));
    return hipGetLastError();
}

template <int S, bool FF, bool W, bool LES, bool VAR>
static hipError_t adjoint_k(const LaunchArgs& a, const void* state, const void* lam_in, void* lam_out, void* grad_F) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    const dim3 grid = grid_for(a.g, bx);
    const auto L = make_launch<R>(a);
    return launch_z_chunks(a.g, grid, true, [&](const dim3& gq, const Geom& gg) {
        k_adjoint<S, FF, W, LES, VAR><<<gq, bx, 0, (hipStream_t)a.stream>>>((const T*)state, (const R*)lam_in, (R*)lam_out,
                                                                            (R*)grad_F, (const R*)a.force_field, gg, L);
    });

}
template <int S, bool FF, bool W>
static hipError_t adjoint_w(const LaunchArgs& a, const void* state, const void* lam_in, void* lam_out, void* grad_F) {
    const bool les = a.cs_smag > 0.0, var = (a.flags & 3u) != 0;
    if (var)
        return les ? adjoint_k<S, FF, W, true, true>(a, state, lam_in, lam_out, grad_F)
                   : adjoint_k<S, FF, W, false, true>(a, state, lam_in, lam_out, grad_F);
    return les ? adjoint_k<S, FF, W, true, false>(a, state, lam_in, lam_out, grad_F)
               : adjoint_k<S, FF, W, false, false>(a, state, lam_in, lam_out, grad_F);
}
template <int S, bool FF>
static hipError_t adjoint_t(const LaunchArgs& a, const void* state, const void* lam_in, void* lam_out, void* grad_F) {
    return a.walls ? adjoint_w<S, FF, true>(a, state, lam_in, lam_out, grad_F)
                   : adjoint_w<S, FF, false>(a, state, lam_in, lam_out, grad_F);
}

template <int S, bool FF>
static hipError_t seed_t(const LaunchArgs& a, const void* state, void* lam_out, void* grad_F) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    const dim3 grid = grid_for(a.g, bx);
    if (a.walls)
        k_energy_seed<S, FF, true><<<grid, bx, 0, (hipStream_t)a.stream>>>((const T*)state, (R*)lam_out, (R*)grad_F,
                                                                           (const R*)a.force_field, a.g, make_launch<R>(a));
    else
        k_energy_seed<S, FF><<<grid, bx, 0, (hipStream_t)a.stream>>>((const T*)state, (R*)lam_out, (R*)grad_F,
                                                                     (const R*)a.force_field, a.g, make_launch<R>(a));
    return hipGetLastError();
}

template <int S, bool W, bool FF>
static hipError_t reduce_t(const LaunchArgs& a, const void* src, double* partial, double* out, size_t max_blocks) {
    using T = typename Store<S>::T;
    using R = typename Store<S>::R;
    int bx;
    dim3 grid = grid_for(a.g, bx);
    const size_t ntiles = (size_t)grid.x * grid.y * grid.z;
    if (max_blocks && ntiles > max_blocks) grid = dim3((unsigned)max_blocks, 1, 1);
    k_reduce_partial<S, W, FF><<<grid, bx, 0, (hipStream_t)a.stream>>>((const T*)src, (const R*)a.force_field, partial,
                                                                      a.g, make_launch<R>(a));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_final(partial, (size_t)grid.x * grid.y * grid.z, out, a.stream);
}

#define CM_DISPATCH_S(fn, ...)                                  \
    switch (a.storage) {                                         \
        case 0: return fn<0>(__VA_ARGS__);                       \
        case 1: return fn<1>(__VA_ARGS__);                       \
        case 2: return fn<2>(__VA_ARGS__);                       \
        case 3: return fn<3>(__VA_ARGS__);                       \
        default: return hipErrorInvalidValue;                    \
    }

template <int S>
static hipError_t init_s(const LaunchArgs& a, void* dst, const void* rho, const void* u, int dt) {
    if (a.walls) return a.force_field ? init_t<S, true, true>(a, dst, rho, u, dt) : init_t<S, true, false>(a, dst, rho, u, dt);
    return a.force_field ? init_t<S, false, true>(a, dst, rho, u, dt) : init_t<S, false, false>(a, dst, rho, u, dt);
}
template <int S>
static hipError_t setpop_s(const LaunchArgs& a, void* dst, const void* f, int dt) {
    return a.walls ? setpop_t<S, true>(a, dst, f, dt) : setpop_t<S, false>(a, dst, f, dt);
}
template <int S>
static hipError_t read_s(const LaunchArgs& a, const void* src, void* o0, void* o1, int dt, int mode) {
    if (a.walls) return a.force_field ? read_t<S, true, true>(a, src, o0, o1, dt, mode) : read_t<S, true, false>(a, src, o0, o1, dt, mode);
    return a.force_field ? read_t<S, false, true>(a, src, o0, o1, dt, mode) : read_t<S, false, false>(a, src, o0, o1, dt, mode);
}
template <int S>
static hipError_t reduce_s(const LaunchArgs& a, const void* src, double* partial, double* out, size_t mb) {
    if (a.walls) return a.force_field ? reduce_t<S, true, true>(a, src, partial, out, mb) : reduce_t<S, true, false>(a, src, partial, out, mb);
    return a.force_field ? reduce_t<S, false, true>(a, src, partial, out, mb) : reduce_t<S, false, false>(a, src, partial, out, mb);
}

}  // namespace cm

// Host-callable launchers (C++ linkage, used by the C ABI layer).
namespace cm {
hipError_t launch_step(const LaunchArgs& a, const void* src, void* dst) { CM_DISPATCH_S(step_w, a, src, dst) }
hipError_t launch_init_equilibrium(const LaunchArgs& a, void* dst, const void* rho, const void* u, int dt) {
    CM_DISPATCH_S(init_s, a, dst, rho, u, dt)
}
hipError_t launch_step_inplace(const LaunchArgs& a, void* buf) { CM_DISPATCH_S(step_inplace_s, a, buf) }
hipError_t launch_set_populations(const LaunchArgs& a, void* dst, const void* f, int dt) {
    CM_DISPATCH_S(setpop_s, a, dst, f, dt)
}
hipError_t launch_read(const LaunchArgs& a, const void* src, void* out0, void* out1, int dt, int mode) {
    CM_DISPATCH_S(read_s, a, src, out0, out1, dt, mode)
}
hipError_t launch_adjoint(const LaunchArgs& a, const void* state, const void* lam_in, void* lam_out, void* grad_F) {
    switch (a.storage) {
        case 0: return a.force_field ? adjoint_t<0, true>(a, state, lam_in, lam_out, grad_F)
                                     : adjoint_t<0, false>(a, state, lam_in, lam_out, grad_F);
        case 1: return a.force_field ? adjoint_t<1, true>(a, state, lam_in, lam_out, grad_F)
                                     : adjoint_t<1, false>(a, state, lam_in, lam_out, grad_F);
        case 2: return a.force_field ? adjoint_t<2, true>(a, state, lam_in, lam_out, grad_F)
                                     : adjoint_t<2, false>(a, state, lam_in, lam_out, grad_F);
        case 3: return a.force_field ? adjoint_t<3, true>(a, state, lam_in, lam_out, grad_F)
                                     : adjoint_t<3, false>(a, state, lam_in, lam_out, grad_F);
        default: return hipErrorInvalidValue;
    }
}
hipError_t launch_energy_seed(const LaunchArgs& a, const void* state, void* lam_out, void* grad_F) {
    switch (a.storage) {
        case 0: return a.force_field ? seed_t<0, true>(a, state, lam_out, grad_F) : seed_t<0, false>(a, state, lam_out, grad_F);
        case 1: return a.force_field ? seed_t<1, true>(a, state, lam_out, grad_F) : seed_t<1, false>(a, state, lam_out, grad_F);
        case 2: return a.force_field ? seed_t<2, true>(a, state, lam_out, grad_F) : seed_t<2, false>(a, state, lam_out, grad_F);
        case 3: return a.force_field ? seed_t<3, true>(a, state, lam_out, grad_F) : seed_t<3, false>(a, state, lam_out, grad_F);
        default: return hipErrorInvalidValue;
    }
}
hipError_t launch_reduce(const LaunchArgs& a, const void* src, double* partial, double* out, size_t max_blocks) {
    CM_DISPATCH_S(reduce_s, a, src, partial, out, max_blocks)
}
hipError_t launch_copy(const void* src, void* dst, size_t bytes, void* stream) {
    const size_t n16 = bytes / 16;
    const size_t blocks = (n16 + 63) / 64;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    k_copy<<<(unsigned)blocks, 64, 0, (hipStream_t)stream>>>((const u32x4*)src, (u32x4*)dst, n16);
    return hipGetLastError();
}
hipError_t launch_reduce_final(const double* partial, size_t nparts, double* out, void* stream) {
    k_reduce_final<<<1, 256, 0, (hipStream_t)stream>>>(partial, nparts, out);
    return hipGetLastError();
}
hipError_t launch_zero(void* dst, size_t bytes, void* stream) {
    const size_t n = bytes / 4;
    const size_t blocks = (n + 255) / 256;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    k_zero<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>((unsigned int*)dst, n);
    return hipGetLastError();
}
// Scratch of the allocation-free reductions: the partials of at most
// kStaticReduceBlocks workgroups (65,536 bytes per device, held until the
// process ends). In host code `scratch` names a
// host-side stand-in, not the device array: its device address comes from
// hipGetSymbolAddress, looked up once per device with that device current.
static __device__ __align__(256) double scratch[8 * kStaticReduceBlocks];

hipError_t static_reduce_scratch(int device, double** ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = (double*)p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

size_t reduce_partials(const Geom& g) {
    int bx;
    const dim3 grid = grid_for(g, bx);
    return (size_t)grid.x * grid.y * grid.z;
}
}  // namespace cm
