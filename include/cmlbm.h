/*
 * cmlbm: cascaded central-moment lattice Boltzmann step on a D3Q27 lattice,
 * hand-written HIP for gfx950 (AMD Instinct MI355X). C ABI.
 *
 * Method: Premnath & Banerjee, "Inertial frame independent forcing for
 * discrete velocity Boltzmann equation: implications for filtered turbulence
 * simulation" (arXiv:1202.6074). The paper derives the scheme for D2Q9; this
 * library implements its three-dimensional generalisation on the
 * tensor-product D3Q27 lattice:
 *   - state: transformed populations fbar = f - S/2 (Sec. 6, Eq. cascadedLBE3);
 *   - moments: rho = sum fbar, rho u = sum fbar e + F/2
 *     (Eqs. densitycalculation, velocitycalculation);
 *   - collision: central moments about u (Eq. binomialtheorem), source
 *     central moments from the exact identity of Sec. 5
 *     (Eq. centralmomentforceexactidentity2) taken order by order (Sec. 8),
 *     relaxation towards the transformed attractor kappa^M - sigma/2
 *     (Eq. centralmomenttransformed) with the rates of Sec. 10
 *     (nu = cs^2 (1/omega_shear - 1/2)), exact return to velocity space;
 *   - streaming: standard (Eq. cascadedstreaming1).
 * Additions not in the paper: Smagorinsky eddy viscosity from the local
 * non-equilibrium second central moments, halfway bounce-back walls, storage
 * shifted by the rest state in FP32/FP16, FP64 reductions, and a discrete
 * adjoint step.
 *
 * Conventions
 *   - Grid nx * ny * nz cells, N = nx*ny*nz < 2^31, ny and nz < 65536; cell
 *     c = x + nx*(y + ny*z). The kernels address a grid row as a pointer plus
 *     a 32-bit byte offset per lane, so 3*nx*E and nx*C must stay below 2^32
 *     (E the storage element size, C the compute type's: nx <= 178,956,970
 *     for FP64, 357,913,941 for FP32 and FP32 shifted, 715,827,882 for FP16
 *     shifted); cmlbm_create rejects longer rows.
 *   - Population index i = (ex+1) + 3(ey+1) + 9(ez+1); opposite is 26 - i.
 *     Weights w_i = w(ex) w(ey) w(ez), w(0) = 2/3, w(+-1) = 1/6.
 *   - Canonical population arrays are structure-of-arrays: 27 planes of N
 *     values, plane i holding population i. Vector fields are 3 planes of N
 *     (x, y, z components); scalars 1 plane of N.
 *   - Time levels: the canonical state fbar(n) is after streaming and before
 *     collision; moments at step n are computed from it. One step maps
 *     fbar(n) to fbar(n+1) (collide, then stream).
 *   - Internally the population buffers hold the post-collision, not yet
 *     streamed values (pull scheme) in a row-interleaved layout: element
 *     (i, x, y, z) at ((z*ny + y)*27 + i)*nx + x. get/set_populations
 *     convert to and from the canonical arrays.
 *
 * D2Q9 (desc.lattice = CMLBM_D2Q9, nz = 1): the lattice on which the paper
 * derives the scheme. Everything above applies with these changes:
 *   - Canonical population arrays have 9 planes in the paper's velocity
 *     order alpha = 0..8: rest, (1,0), (0,1), (-1,0), (0,-1), (1,1), (-1,1),
 *     (-1,-1), (1,-1) (Sec. 2); w = 4/9, 1/9 (axes), 1/36 (diagonals).
 *   - Vector fields (u, force field) have 2 planes (x, y); the third
 *     component of the uniform force and of the wall velocities is ignored;
 *     cmlbm_reduce reports momentum z = 0.
 *   - Rates in the paper's numbering (Sec. 10): omega_bulk = omega_3 (trace
 *     of the second-order moments), omega_shear = omega_4 = omega_5,
 *     omega3[0] = omega_6 (xxy), omega3[1] = omega_7 (xyy),
 *     omega4[0] = omega_8 (xxyy); omega3[2], omega4[1], omega5 and omega6
 *     are validated but unused. The eddy viscosity and all three flags
 *     apply (the sub-grid stress has 3 planes: xx, yy, xy).
 *   - Internal layout (y*9 + i)*nx + x with i = (ex+1) + 3(ey+1); buffers
 *     need 9*N elements.
 *   - cmlbm_adjoint_step and cmlbm_energy_seed return CMLBM_EINVAL.
 *
 * Memory and ownership
 *   - Every pointer argument is a DEVICE pointer unless marked [host].
 *   - The caller allocates and owns the two population buffers, the force
 *     field, the moment/population output arrays and the adjoint arrays;
 *     they must outlive the handle. The library allocates only a small
 *     device scratch area for reduction partials, freed by cmlbm_destroy
 *     (cmlbm_reduce_noalloc uses a static device array instead).
 *   - All work is enqueued on the HIP stream given at creation. Functions
 *     return after enqueueing, except cmlbm_reduce, which synchronises the
 *     stream to return its host result.
 *
 * Errors
 *   - Every function returns a cmlbm_status; nothing throws, exits or aborts.
 *   - Arguments are validated on the host before any launch (CMLBM_EINVAL).
 *   - HIP launch errors return CMLBM_EHIP; asynchronous device errors surface
 *     at the next synchronising call (cmlbm_reduce) as CMLBM_EHIP.
 *   - cmlbm_last_error() returns a thread-local message for the last failure.
 */
#ifndef CMLBM_H
#define CMLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cmlbm_lattice* cmlbm_handle;

typedef enum {
    CMLBM_OK = 0,
    CMLBM_EINVAL = 1,      /* invalid argument (checked on the host)            */
    CMLBM_ENOMEM = 2,      /* scratch allocation failed                          */
    CMLBM_EHIP = 3,        /* HIP runtime error                                  */
    CMLBM_ENONFINITE = 4,  /* reduction found non-finite rho or u                */
    CMLBM_ESTATE = 5       /* call not valid in the current state                */
} cmlbm_status;

/* Population storage. The compute type is FP64 for CMLBM_F64 and FP32
 * otherwise. Shifted modes store fbar_i - w_i rho0 (IEEE binary32 or
 * binary16, round to nearest even). */
typedef enum {
    CMLBM_F64 = 0,
    CMLBM_F32 = 1,
    CMLBM_F32_SHIFTED = 2,
    CMLBM_F16_SHIFTED = 3
} cmlbm_storage;

/* Lattice model. CMLBM_D2Q9 is the two-dimensional lattice of the paper
 * (Sec. 2), on a grid with nz = 1; see "D2Q9" below. */
typedef enum { CMLBM_D3Q27 = 0, CMLBM_D2Q9 = 1 } cmlbm_lattice_kind;

/* Streaming scheme. Two buffers: pull scheme alternating between buf_a and
 * buf_b. In place (D3Q27): one buffer (buf_b null) updated by alternating
 * even and odd steps (the AA pattern); half the memory, the same bytes per
 * update and bitwise the same results. With in-place streaming the meaning
 * of the buffer depends on the parity of the steps taken since the state was
 * set, cmlbm_step_from, the adjoint and the sub-grid force are unavailable
 * (CMLBM_EINVAL), and a copy of cmlbm_state_buffer may only be restored at
 * the same parity; cmlbm_get/set_populations are the portable checkpoint. */
typedef enum { CMLBM_STREAM_TWO_BUFFERS = 0, CMLBM_STREAM_IN_PLACE = 1 } cmlbm_streaming;

/* Element type of caller arrays exchanged with the library. */
typedef enum { CMLBM_DT_F64 = 0, CMLBM_DT_F32 = 1 } cmlbm_dtype;

typedef struct {
    int32_t nx, ny, nz;     /* grid size, each >= 1                              */
    int32_t storage;        /* cmlbm_storage                                     */
    uint32_t walls;         /* bit 0: halfway bounce-back planes at y = -1/2 and
                               y = ny - 1/2 (x and z stay periodic); 0: periodic */
    uint32_t tuning;        /* performance hints (results are identical):
                               bits 0-1 must be 0; bits above 7 too;
                               bit 2: one block per grid row in the step
                               kernel (looping over x); bits 3-4 workgroup
                               order of the step kernel: 0 library default
                               (XCD-aware for FP64 storage and when a row
                               spans several workgroups, nx > 256 without
                               bit 2; runs of 32 for periodic D3Q27 FP32 and
                               FP32-shifted rows of 129-256 cells without
                               bit 2, except the sub-grid-force step; runs of
                               256 for FP16 rows of the two-cells-per-lane
                               kernel; plain otherwise), 1
                               plain, 2 XCD-aware (each XCD takes a
                               contiguous range of rows), 3 runs of 32
                               consecutive workgroups per XCD in turn
                               (orders whose workgroup count is not a
                               multiple of 8, resp. 256, fall back to
                               plain);
                               bit 5: per-lane shifted loads in the step
                               kernel also where one workgroup covers a row
                               (no LDS exchange; also no two-cell FP16
                               kernel); bit 6: FP16 storage, one cell per lane
                               also on even rows of at most 512 cells (no
                               two-cell kernel); bit 7: every step and
                               adjoint step in one launch (by default the
                               FP32 and FP32-shifted step with one workgroup
                               per row, and the adjoint step, run over
                               chunks of 128 z-planes); 0 = defaults          */
    double wall_u_lo[3];    /* velocity of the wall at y = -1/2                  */
    double wall_u_hi[3];    /* velocity of the wall at y = ny - 1/2              */
    double rho0;            /* reference density (rest state, wall density) > 0  */
    int32_t lattice;        /* cmlbm_lattice_kind                                */
    uint32_t streaming;     /* cmlbm_streaming                                   */
} cmlbm_desc;

/* Relaxation rates, each in (0, 2). omega_shear and omega_bulk are the
 * second-order deviatoric and trace rates (Sec. 10: omega_4 = omega_5 and
 * omega_3 of the paper); nu = (1/omega_shear - 1/2)/3. Higher-order rates
 * are free: omega3 = {(xyy+xzz)-type, (xyy-xzz)-type, xyz},
 * omega4 = {xxyy-type, xxyz-type}, omega5 (fifth order), omega6 (xxyyzz).
 * cs_smag >= 0 is the Smagorinsky constant (0 disables the eddy viscosity;
 * filter width one cell). flags: bit 0 CMLBM_FACTORIZED, fourth- and
 * sixth-order attractors as products of the post-collision second-order
 * central moments (Sec. 13); bit 1 CMLBM_REDUCED_COMPRESSIBILITY,
 * rho0 u = sum fbar e + F/2 (Sec. 12; moments, reductions and the initial
 * state follow the same definition); bit 2 CMLBM_SGS_FORCE, the sub-grid
 * stresses act as a force instead of an eddy viscosity in the collision
 * (Sec. 14, see cmlbm_set_sgs_buffers; periodic lattices). reserved
 * must be 0. */
#define CMLBM_FACTORIZED 1u
#define CMLBM_REDUCED_COMPRESSIBILITY 2u
#define CMLBM_SGS_FORCE 4u
typedef struct {
    double omega_shear, omega_bulk;
    double omega3[3];
    double omega4[2];
    double omega5, omega6;
    double cs_smag;
    uint32_t flags;
    uint32_t reserved;
} cmlbm_relax;

/* Create a lattice: the grid, the populations fbar of Sec. 6
 * (Eq. cascadedLBE3) in the chosen storage, and the streaming scheme of
 * Eq. cascadedstreaming1. buf_a and buf_b are two device buffers of
 * bytes_each >= Q*N*element bytes (Q = 27 for D3Q27, 9 for D2Q9; element 8,
 * 4, 4, 2 bytes for the storage modes), caller-owned and borrowed for the
 * handle's lifetime; hip_stream is a hipStream_t (may be null for the default
 * stream). Every description field is validated on the host (CMLBM_EINVAL,
 * nothing allocated); then a small device scratch area for the reductions is
 * allocated (CMLBM_EHIP on failure). Relaxation defaults to omega_shear = 1
 * and all other rates 1, no eddy viscosity, F = 0. The state is undefined
 * until cmlbm_init_equilibrium or cmlbm_set_populations. */
cmlbm_status cmlbm_create(const cmlbm_desc* desc /* [host] */, void* buf_a, void* buf_b, size_t bytes_each,
                          void* hip_stream, cmlbm_handle* out /* [host] */);
/* Synchronises the handle's stream, frees the reduction scratch and the
 * handle (null is accepted). Caller buffers are not touched. */
cmlbm_status cmlbm_destroy(cmlbm_handle h);

/* Change the stream later work is enqueued on. */
cmlbm_status cmlbm_set_stream(cmlbm_handle h, void* hip_stream);

/* Relaxation rates of Sec. 10 (Eq. cascadedcollision1 relaxes each central
 * moment group with its rate), the Smagorinsky constant and the flags above.
 * Every field is validated before the handle (CMLBM_EINVAL: a rate outside
 * (0, 2), cs_smag < 0 or non-finite, undefined flags or reserved != 0;
 * CMLBM_SGS_FORCE on a walled or in-place lattice). Takes effect from the
 * next launch. */
cmlbm_status cmlbm_set_relaxation(cmlbm_handle h, const cmlbm_relax* relax /* [host] */);

/* Body force (Sec. 3). uniform [host] is used when field is null; field is a
 * 3*N structure-of-arrays device array in the compute type (double for
 * CMLBM_F64, float otherwise), borrowed until replaced. */
cmlbm_status cmlbm_set_force(cmlbm_handle h, const double uniform[3], const void* field);

/* Initial state whose central moments are the transformed attractor
 * kappa^M - sigma/2 (Eq. centralmomenttransformed, with the Maxwellian
 * central moments of Eq. centralmomentMaxwelldistribution and the source
 * moments of Sec. 8) at the given rho and u, so that rho and u read back
 * exactly through Eqs. densitycalculation and velocitycalculation.
 * rho: N values or null (rho0 everywhere); u: 3*N values (2*N on D2Q9);
 * both device arrays of type dt, read before the next call on the stream
 * returns its work. Uses the force set by cmlbm_set_force. Errors:
 * CMLBM_EINVAL for a null u or unknown dt, CMLBM_EHIP for a launch failure. */
cmlbm_status cmlbm_init_equilibrium(cmlbm_handle h, const void* rho, const void* u, cmlbm_dtype dt);

/* Advance nsteps >= 0 steps, each the collision of Eq. cascadedcollision1
 * (central moments about u, source moments of Sec. 8, relaxation with the
 * rates of Sec. 10) followed by the streaming of Eq. cascadedstreaming1,
 * alternating buffers (or in place). Enqueued on the stream; CMLBM_EINVAL for
 * nsteps < 0, CMLBM_ESTATE when the sub-grid force lacks its buffers,
 * CMLBM_EHIP for a launch failure (steps launched before it stay queued). */
cmlbm_status cmlbm_step(cmlbm_handle h, int64_t nsteps);

/* One step (Eqs. cascadedcollision1, cascadedstreaming1) from the
 * internal-layout buffer src into dst (both Q*N elements of the storage type;
 * may be the handle's own buffers or caller stash buffers, but must not alias
 * each other). The handle's state is unchanged. CMLBM_EINVAL for null or
 * equal buffers, with the sub-grid force or with in-place streaming. */
cmlbm_status cmlbm_step_from(cmlbm_handle h, const void* src, void* dst);

/* Device pointer of the buffer holding the current state fbar(n)
 * (Eq. cascadedLBE3) in the internal layout (for device-to-device
 * checkpoints), and its size in bytes (bytes may be null). */
cmlbm_status cmlbm_state_buffer(cmlbm_handle h, void** buf /* [host] */, size_t* bytes /* [host] */);

/* rho = sum fbar (Eq. densitycalculation) and u = (sum fbar e + F/2)/rho
 * (Eq. velocitycalculation; Eq. resolvedvelocitycalculation with the
 * sub-grid force) at the current step, from the pre-collision fbar(n).
 * rho: N device values, u: 3*N (2*N for D2Q9), type dt, overwritten.
 * CMLBM_EINVAL for null arrays or an unknown dt. */
cmlbm_status cmlbm_read_moments(cmlbm_handle h, void* rho, void* u, cmlbm_dtype dt);

/* The state fbar(n) = f - S/2 of Eq. cascadedLBE3 (after streaming, before
 * collision) as Q*N canonical device values of type dt (unshifted: the rest
 * state w_i rho0 included), read (get) or replaced (set). The conversion to
 * and from the internal layout applies the streaming permutation, a
 * bijection also with bounce-back walls. set also resets the sub-grid
 * stress. CMLBM_EINVAL for a null f or an unknown dt. */
cmlbm_status cmlbm_get_populations(cmlbm_handle h, void* f, cmlbm_dtype dt);
cmlbm_status cmlbm_set_populations(cmlbm_handle h, const void* f, cmlbm_dtype dt);

/* FP64 reductions over the current state, deterministic (fixed-order tree),
 * of rho and u as Eqs. densitycalculation and velocitycalculation define them:
 * out[8] [host] = {mass, momentum x, y, z (sum rho u), kinetic energy
 * sum rho|u|^2/2, number of cells with non-finite rho or u, min rho,
 * max |u|}. Synchronises the stream. Returns CMLBM_ENONFINITE (with out
 * filled) when out[5] > 0, CMLBM_EHIP for a device error (also one left by
 * earlier asynchronous work). */
cmlbm_status cmlbm_reduce(cmlbm_handle h, double out[8]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * reductions of cmlbm_reduce, enqueued on the handle's stream without
 * allocating, without copying to the host and without synchronising.
 * out: DEVICE array of 8 doubles, overwritten with the same quantities as
 * cmlbm_reduce's out (non-finite cells are counted in out[5]; the status does
 * not report them, since nothing is read back). The results equal
 * cmlbm_reduce's up to FP64 rounding (the cells are summed in another
 * order), and are themselves deterministic.
 * Scratch: a static device array of CMLBM_REDUCE_NOALLOC_SCRATCH_BYTES that
 * each device holds from the first call on it until the process ends; the
 * partial-sum kernel launches at most 1024 workgroups, each combining several
 * row chunks, so every lattice size fits and no size is rejected. Every call
 * on one device shares that device's array and leaves its partial sums there
 * (each slot is written before it is read, so nothing needs clearing): calls
 * that overlap in time on one device (several streams or threads) race and
 * must be serialised by the caller. Errors: CMLBM_EINVAL for a null out,
 * CMLBM_ESTATE as cmlbm_reduce, CMLBM_EHIP for a launch failure or a failed
 * lookup of the static array. */
#define CMLBM_REDUCE_NOALLOC_SCRATCH_BYTES 65536
cmlbm_status cmlbm_reduce_noalloc(cmlbm_handle h, double* out);

/* Discrete adjoint of one step (project addition: the transpose of the
 * linearised collision of Eq. cascadedcollision1 and of the streaming of
 * Eq. cascadedstreaming1; periodic or walled lattices, the bounce-back
 * transposed: lambda of a population that returns from a wall feeds the
 * opposite population of the same cell; every storage mode: the state is
 * read as stored and the collision linearised in the compute type at those
 * values, the rounding to the storage type not being differentiated).
 * With cs_smag > 0 the collision's shear rate is the eddy rate of the
 * Smagorinsky model, a function of the cell's second-order central moments,
 * and the adjoint differentiates through it; its norm
 * Q = sqrt(2 Pi^d : Pi^d) has no derivative at Q = 0, where it is taken as 0
 * (the rate is then omega_shear to first order). state: internal-layout
 * buffer whose gather is fbar(n) (the buffer the forward step n read);
 * lam_in: dL/dfbar(n+1), lam_out: dL/dfbar(n), 27*N each in the row layout
 * of the population buffers, element (i, x, y, z) at ((z*ny + y)*27 + i)*nx
 * + x (the canonical population index i of fbar, not permuted by the
 * streaming); grad_F: 3*N accumulator in the force field's layout,
 * grad_F += dL/dF through step n. Arrays are in the compute type. lam_in and
 * lam_out must not alias. The factorized attractors and reduced
 * compressibility (Secs. 12-13) are differentiated too; the sub-grid stress
 * as a force is not (CMLBM_EINVAL). */
cmlbm_status cmlbm_adjoint_step(cmlbm_handle h, const void* state, const void* lam_in, void* lam_out, void* grad_F);

/* Seeds for the loss E = sum_x rho |u|^2 / 2 at the state held in `state`,
 * with rho and u of Eqs. densitycalculation and velocitycalculation:
 * lam_out = dE/dfbar = u.e_i - |u|^2/2 (27*N, in the row layout of
 * cmlbm_adjoint_step), grad_F = dE/dF = u/2 (3*N, overwritten); with reduced
 * compressibility (Sec. 12: rho0 u = sum fbar e + F/2, E as cmlbm_reduce
 * computes it) dE/dfbar = (rho/rho0) u.e_i + |u|^2/2, dE/dF = (rho/rho0) u/2.
 * Same conditions as cmlbm_adjoint_step. */
cmlbm_status cmlbm_energy_seed(cmlbm_handle h, const void* state, void* lam_out, void* grad_F);

/* Sub-grid stresses as a force (Sec. 14; relaxation flag CMLBM_SGS_FORCE).
 * The filtered equation of Sec. 14 feels the unresolved motion as the
 * acceleration a' = -div R: the source central moments follow the exact
 * identity with a' in place of F/rho, and the momentum takes rho a'/2
 * (Eq. resolvedvelocitycalculation). The closure of R is not fixed by the
 * paper; the library uses Smagorinsky for its deviatoric part,
 * R^d = -2 C_s^2 |S| S (C_s = cs_smag, filter width one cell), with the strain
 * rate from the pre-collision non-equilibrium second central moments,
 * S = -omega_shear Pi^d / (2 rho cs^2) (rho0 with reduced compressibility),
 * and a'(n) = -div R(n-1) by second-order central differences (the stress of
 * the previous step: one step of lag keeps the step explicit). The force of
 * step n is then F + rho(n) a'(n); moments and reductions include it. The
 * collision keeps omega_shear (no eddy rate).
 * stress_a and stress_b: two distinct device buffers of bytes_each >= 6*N
 * values of the compute type (double for CMLBM_F64, float otherwise), caller
 * owned, planes xx, yy, zz, xy, xz, yz (structure of arrays, cell order as
 * the populations); on D2Q9 3*N values, planes xx, yy, xy. Buffer k holds the stress that belongs to population
 * buffer k; both are zeroed here and by cmlbm_init_equilibrium and
 * cmlbm_set_populations (a new state starts without sub-grid force). With
 * the flag set, cmlbm_step, cmlbm_read_moments and cmlbm_reduce return
 * CMLBM_ESTATE until the buffers are given; cmlbm_step_from returns
 * CMLBM_EINVAL (it does not carry the stress), and so does in-place streaming. */
cmlbm_status cmlbm_set_sgs_buffers(cmlbm_handle h, void* stress_a, void* stress_b, size_t bytes_each);

/* Measurement utility: plain device-to-device copy of `bytes` (a multiple of
 * 16; both addresses 16-byte aligned) with a streaming kernel, enqueued on
 * hip_stream. Used as the reference for achievable HBM bandwidth and to
 * calibrate hardware byte counters; not part of the method. */
cmlbm_status cmlbm_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

/* Thread-local description of the last error (never null). */
const char* cmlbm_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t cmlbm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CMLBM_H */
