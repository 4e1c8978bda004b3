// Host-side interface between the C ABI layer and the device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cm {

struct Geom {
    int nx, ny, nz;
    int64_t N;     // nx * ny * nz (< 2^31, checked by the caller)
    int rowloop;   // step kernel: 1 = one block per grid row, looping over x
    int lanegather;   // step kernel: 1 = per-lane shifted loads also where one workgroup covers a row
    int pairs_off;    // step kernel: 1 = one cell per lane also for FP16 rows (no two-cell kernel)
    int one_launch;   // step kernel: 1 = all z-planes in one launch (no chunks of planes)
    int xcd;       // step kernel workgroup order: 0 plain, 1 XCD-aware (contiguous eighths),
                   // R >= 2 runs of R consecutive workgroups per XCD in turn (block_coords)
    int aa;        // streaming: 0 two buffers (pull); in place: 1 even parity (natural), 2 odd parity
    // rows of a step launch: y = ybase + ystride * (row index), yrows of them
    // (all rows by default; the interior and the two wall rows are launched
    // separately when there are walls)
    int ybase, ystride, yrows;
    int zbase;     // first z-plane of this launch (launches over chunks of planes)
};

struct LaunchArgs {
    Geom g;
    int lattice;          // 0 D3Q27, 1 D2Q9 (nz = 1)
    int storage;          // 0 f64, 1 f32, 2 f32 shifted, 3 f16 shifted
    int walls;            // halfway bounce-back planes at y = -1/2, ny - 1/2
    double rho0;
    double omega_shear, omega_bulk, omega3[3], omega4[2], omega5, omega6;
    double cs_smag;
    int xcd_default;      // 1: g.xcd is the library's default, not the caller's hint
    unsigned flags;       // bit 0: factorized attractors, bit 1: reduced compressibility
    double force[3];            // uniform force (when force_field is null)
    const void* force_field;    // 3*N SoA in the compute type, or null
    double wall_u_lo[3], wall_u_hi[3];
    void* stream;
    // sub-grid stress as a force (flags bit 2): stress of the previous step
    // (read) and of this step (written), 6 planes of N in the compute type
    const void* stress_prev;
    void* stress_next;
};

hipError_t launch_step(const LaunchArgs& a, const void* src, void* dst);
// in-place streaming: one step on the single buffer, even or odd kernel by a.g.aa
hipError_t launch_step_inplace(const LaunchArgs& a, void* buf);
hipError_t launch_init_equilibrium(const LaunchArgs& a, void* dst, const void* rho, const void* u, int dt);
hipError_t launch_set_populations(const LaunchArgs& a, void* dst, const void* f, int dt);
// mode 0: canonical populations into out0; mode 1: rho into out0, u into out1
hipError_t launch_read(const LaunchArgs& a, const void* src, void* out0, void* out1, int dt, int mode);
hipError_t launch_adjoint(const LaunchArgs& a, const void* state, const void* lam_in, void* lam_out, void* grad_F);
hipError_t launch_energy_seed(const LaunchArgs& a, const void* state, void* lam_out, void* grad_F);
// FP64 reductions into out[8] (device). The partial kernel writes 8 doubles per
// workgroup into `partial`: with max_blocks = 0 one workgroup per tile (a
// workgroup-wide chunk of a grid row, reduce_partials(g) of them); otherwise at
// most max_blocks workgroups, each combining several tiles, so that `partial`
// needs 8 * min(max_blocks, reduce_partials(g)) doubles.
hipError_t launch_reduce(const LaunchArgs& a, const void* src, double* partial, double* out, size_t max_blocks = 0);
hipError_t launch_reduce_final(const double* partial, size_t nparts, double* out, void* stream);
size_t reduce_partials(const Geom& g);
// Reductions without allocation: the partials go to a static device array of
// 8 * kStaticReduceBlocks doubles per device. static_reduce_scratch gives its
// address on `device`, looked up once per device and cached.
constexpr size_t kStaticReduceBlocks = 1024;
hipError_t static_reduce_scratch(int device, double** ptr);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, void* stream);
// zero `bytes` (a multiple of 4) with a fill kernel
hipError_t launch_zero(void* dst, size_t bytes, void* stream);

}  // namespace cm

// D2Q9 launchers (same arguments; vector arrays have 2 planes, population
// arrays 9 planes in the paper's velocity order).
namespace cm2 {
hipError_t launch_step(const cm::LaunchArgs& a, const void* src, void* dst);
hipError_t launch_init_equilibrium(const cm::LaunchArgs& a, void* dst, const void* rho, const void* u, int dt);
hipError_t launch_set_populations(const cm::LaunchArgs& a, void* dst, const void* f, int dt);
hipError_t launch_read(const cm::LaunchArgs& a, const void* src, void* out0, void* out1, int dt, int mode);
hipError_t launch_reduce(const cm::LaunchArgs& a, const void* src, double* partial, double* out, size_t max_blocks = 0);
}  // namespace cm2
