// Device helpers shared by the D3Q27 and D2Q9 kernels: storage types of the
// population buffers, reading caller arrays of either dtype, and the
// fixed-order FP64 block reduction.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cm {

// Storage mode S: element type T in memory, compute type R, and whether the
// stored value is shifted by the rest state w_i rho0.
template <int S> struct Store;
template <> struct Store<0> { using T = double;   using R = double; static constexpr bool shifted = false; };
template <> struct Store<1> { using T = float;    using R = float;  static constexpr bool shifted = false; };
template <> struct Store<2> { using T = float;    using R = float;  static constexpr bool shifted = true; };
template <> struct Store<3> { using T = _Float16; using R = float;  static constexpr bool shifted = true; };

// Coordinates (x block, y, z) of this workgroup in a grid of (gx, ny, nz)
// blocks. Consecutive workgroups are dispatched round-robin to the eight
// XCDs, each with its own L2. xcd = 0: that order (block k on XCD k % 8);
// xcd = 1: XCD k takes the k-th contiguous eighth of the blocks (in x, y, z
// order), so that rows that share data (x-halo cache lines, neighbouring
// stress rows) are read through one L2; xcd = R >= 2: runs of R consecutive
// blocks go to the XCDs in turn (8 R blocks per round). Orders whose block
// count does not divide fall back to the plain one. Any bijection is correct;
// this one only changes which L2 serves a block and when.
__device__ __forceinline__ void block_coords(int xcd, int& bx, int& y, int& z) {
    const uint32_t gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
    uint32_t lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const uint32_t total = gx * gy * gz;
    if (xcd == 1 && (total & 7u) == 0u) {
        lin = (lin & 7u) * (total >> 3) + (lin >> 3);
    } else if (xcd >= 2 && total % (8u * (uint32_t)xcd) == 0u) {
        const uint32_t run = (uint32_t)xcd, round = lin / (8u * run), k = lin % (8u * run);
        lin = round * 8u * run + (k & 7u) * run + (k >> 3);
    }
    bx = (int)(lin % gx);
    const uint32_t r = lin / gx;
    y = (int)(r % gy);
    z = (int)(r / gy);
}

__device__ __forceinline__ double as_double(const void* p, int dt, size_t k) {
    return dt == 0 ? static_cast<const double*>(p)[k] : static_cast<double>(static_cast<const float*>(p)[k]);
}

// Per-block partials: [mass, px, py, pz, ke, nonfinite, min rho, max |u|], in
// a fixed order so that results are bitwise reproducible.
__device__ __forceinline__ void combine(double (&a)[8], const double (&b)[8]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) a[k] += b[k];
    a[6] = fmin(a[6], b[6]);
    a[7] = fmax(a[7], b[7]);
}

__device__ __forceinline__ void block_reduce(double (&v)[8], double* __restrict__ out) {
    __shared__ double sm[8][256];
    const int t = threadIdx.x + blockDim.x * threadIdx.y;
    const int nt = blockDim.x * blockDim.y;
#pragma unroll
    for (int k = 0; k < 8; ++k) sm[k][t] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s && t + s < nt) {
            double a[8], b[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) { a[k] = sm[k][t]; b[k] = sm[k][t + s]; }
            combine(a, b);
#pragma unroll
            for (int k = 0; k < 8; ++k) sm[k][t] = a[k];
        }
        __syncthreads();
    }
    if (t == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) out[k] = sm[k][0];
    }
}

}  // namespace cm
