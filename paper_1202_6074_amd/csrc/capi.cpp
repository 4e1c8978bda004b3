// C ABI of the cmlbm library: handle management, host-side validation, buffer
// alternation and error reporting. Device work lives in kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/cmlbm.h"
#include "kernels.hpp"

struct cmlbm_lattice {
    cm::LaunchArgs a;
    void* buf[2];
    int cur;             // index of the buffer holding the current state
    size_t bytes_each;
    double* scratch;     // reduction partials followed by 8 result slots
    size_t nparts;
    void* stress[2];     // sub-grid stress buffers (caller-owned); stress[k] pairs with buf[k]
    size_t stress_bytes;
    int device;          // device current at creation (the handle's work runs there)
};

namespace {

thread_local std::string g_err = "no error";

cmlbm_status fail(cmlbm_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

cmlbm_status hip_fail(hipError_t e, const char* where) {
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return CMLBM_EHIP;
}

size_t elem_size(int storage) {
    switch (storage) {
        case CMLBM_F64: return 8;
        case CMLBM_F32: return 4;
        case CMLBM_F32_SHIFTED: return 4;
        case CMLBM_F16_SHIFTED: return 2;
        default: return 0;
    }
}

// Bytes of the compute type (force field, sub-grid stress, adjoint arrays).
size_t compute_size(int storage) { return storage == CMLBM_F64 ? 8 : 4; }

// Largest per-lane byte offset, plus one element, that the kernels form within
// one grid row. Every kernel addresses an element as a workgroup-uniform row
// pointer plus a per-lane 32-bit byte offset: up to three consecutive
// population rows of the internal layout (the three e_x of a gather or an odd
// in-place push, 3 nx elements of the storage type), or one row of a
// compute-type array (force field, sub-grid stress, adjoint arrays). Offsets
// must not wrap, so this span must stay below 2^32.
uint64_t lane_span(int32_t nx, int storage) {
    const uint64_t n = (uint64_t)(nx > 0 ? nx : 0);
    const uint64_t pop = 3 * n * (uint64_t)elem_size(storage), cmp = n * (uint64_t)compute_size(storage);
    return pop > cmp ? pop : cmp;
}

// Populations per cell of the lattice model.
int lattice_q(int lattice) { return lattice == CMLBM_D2Q9 ? 9 : 27; }

bool rate_ok(double w) { return std::isfinite(w) && w > 0.0 && w < 2.0; }

// Workgroup order chosen when the caller gives no hint. When a grid row spans
// several workgroups (nx > 256 without the row loop), the plain order sends
// neighbouring workgroups of one row to different XCDs, whose L2s then fetch
// the cache lines shared at the block boundary twice (and, in the odd
// in-place step, both write parts of the same lines). Measured on MI355X
// (MLUPS, plain / XCD-aware): FP32 512^3 26,002 / 27,664; FP32 1024^3 in place
// 21,423 / 27,103; FP64 512^3 11,539 / 13,311. With one 256-lane workgroup per
// row (periodic D3Q27, FP32 and FP32-shifted rows of 129-256 cells) runs of
// 32 rows per XCD in turn (at 256^3 the eight runs of a round cover one
// z-plane) beat both; measured on four machines at 256^3 (us per step, plain /
// XCD-aware / runs): two-buffer step 602 / 627 / 594, 614 / - / 604,
// 603 / - / 594, 599 / 624 / 591; in place 661 / 673 / 645, 661 / - / 645,
// 660 / - / 644; FP32 shifted 605 / - / 592. Not faster, so kept plain: walls
// (plain / runs 593 / 596 us), rows of 128 cells (77.4 / 78.0 us at 128^3),
// FP16 storage (plain / XCD-aware at 256^3: 329 / 330 us, in place 362 / 373).
// The two-cells-per-lane FP16 kernel (even rows of 258-512 cells, one
// workgroup per row) prefers runs of 256 rows to the XCD-aware order (512^3,
// us per step on three machines: 2742 / 2615 (runs of 512), 2744 / 2722,
// 2750 / 2715).
constexpr int kXcdRun = 32, kXcdRunPairs = 256;
int default_xcd_order(int lattice, int storage, int nx, bool rowloop, bool walls, bool pair_kernel) {
    if (lattice == CMLBM_D3Q27 && storage == CMLBM_F16_SHIFTED && pair_kernel && !rowloop && nx % 2 == 0 &&
        nx > 256 && nx <= 512)
        return kXcdRunPairs;
    if (storage == CMLBM_F64 || (!rowloop && nx > 256)) return 1;
    const bool four_byte = storage == CMLBM_F32 || storage == CMLBM_F32_SHIFTED;
    return lattice == CMLBM_D3Q27 && four_byte && !rowloop && !walls && nx > 128 ? kXcdRun : 0;
}

cmlbm_status check_handle(cmlbm_handle h) {
    if (!h) return fail(CMLBM_EINVAL, "null handle");
    return CMLBM_OK;
}

cmlbm_status check_dtype(cmlbm_dtype dt) {
    if (dt != CMLBM_DT_F64 && dt != CMLBM_DT_F32) return fail(CMLBM_EINVAL, "dtype must be CMLBM_DT_F64 or CMLBM_DT_F32");
    return CMLBM_OK;
}

// Point the launch arguments at the stress buffers paired with the current
// state (read) and the next one (written); null when the sub-grid force is off.
void bind_stress(cmlbm_lattice* h) {
    const bool on = (h->a.flags & CMLBM_SGS_FORCE) != 0;
    h->a.stress_prev = on ? h->stress[h->cur] : nullptr;
    h->a.stress_next = on ? h->stress[h->cur ^ 1] : nullptr;
}

cmlbm_status check_sgs_ready(cmlbm_lattice* h) {
    if ((h->a.flags & CMLBM_SGS_FORCE) && !h->stress[0])
        return fail(CMLBM_ESTATE, "the sub-grid force needs stress buffers (cmlbm_set_sgs_buffers)");
    return CMLBM_OK;
}

// A new state starts with zero sub-grid stress (no force from the previous step).
hipError_t reset_stress(cmlbm_lattice* h) {
    if (!h->stress[0]) return hipSuccess;
    hipError_t e = cm::launch_zero(h->stress[0], h->stress_bytes, h->a.stream);
    if (e == hipSuccess) e = cm::launch_zero(h->stress[1], h->stress_bytes, h->a.stream);
    return e;
}

}  // namespace

extern "C" {

int32_t cmlbm_version(void) { return 10000; }

const char* cmlbm_last_error(void) { return g_err.c_str(); }

cmlbm_status cmlbm_create(const cmlbm_desc* d, void* buf_a, void* buf_b, size_t bytes_each, void* hip_stream,
                          cmlbm_handle* out) {
    if (!d || !out) return fail(CMLBM_EINVAL, "desc and out must be non-null");
    *out = nullptr;
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(CMLBM_EINVAL, "nx, ny, nz must be >= 1");
    if (d->lattice != CMLBM_D3Q27 && d->lattice != CMLBM_D2Q9) return fail(CMLBM_EINVAL, "unknown lattice");
    if (d->lattice == CMLBM_D2Q9 && d->nz != 1) return fail(CMLBM_EINVAL, "D2Q9 requires nz == 1");
    if (d->streaming != CMLBM_STREAM_TWO_BUFFERS && d->streaming != CMLBM_STREAM_IN_PLACE)
        return fail(CMLBM_EINVAL, "desc.streaming must be CMLBM_STREAM_TWO_BUFFERS or CMLBM_STREAM_IN_PLACE");
    const bool inplace = d->streaming == CMLBM_STREAM_IN_PLACE;
    if (inplace && d->lattice != CMLBM_D3Q27) return fail(CMLBM_EINVAL, "in-place streaming is implemented for D3Q27");
    const int64_t N = (int64_t)d->nx * d->ny * d->nz;
    if (N >= ((int64_t)1 << 31)) return fail(CMLBM_EINVAL, "nx*ny*nz must be < 2^31");
    if (d->ny >= 65536 || d->nz >= 65536) return fail(CMLBM_EINVAL, "ny and nz must be < 65536");
    const size_t es = elem_size(d->storage);
    if (!es) return fail(CMLBM_EINVAL, "unknown storage mode");
    if (lane_span(d->nx, d->storage) > 0xffffffffull) {
        char msg[200];
        std::snprintf(msg, sizeof msg,
                      "nx = %d too large for this storage: the kernels address a row with 32-bit byte offsets "
                      "(3*nx*%zu and nx*%zu bytes must stay below 2^32)",
                      d->nx, es, compute_size(d->storage));
        return fail(CMLBM_EINVAL, msg);
    }
    if (d->walls & ~1u) return fail(CMLBM_EINVAL, "walls: only bit 0 is defined");
    if (d->tuning & ~252u) return fail(CMLBM_EINVAL, "tuning: only bits 2-7 are defined");
    if (!(std::isfinite(d->rho0) && d->rho0 > 0)) return fail(CMLBM_EINVAL, "rho0 must be finite and > 0");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(d->wall_u_lo[k]) || !std::isfinite(d->wall_u_hi[k]))
            return fail(CMLBM_EINVAL, "wall velocities must be finite");
    if (inplace) {
        if (!buf_a || buf_b) return fail(CMLBM_EINVAL, "in-place streaming takes one buffer (buf_b must be null)");
    } else if (!buf_a || !buf_b || buf_a == buf_b) {
        return fail(CMLBM_EINVAL, "two distinct non-null buffers are required");
    }
    const size_t need = (size_t)lattice_q(d->lattice) * (size_t)N * es;
    if (bytes_each < need) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "buffers too small: %zu bytes given, %zu needed", bytes_each, need);
        return fail(CMLBM_EINVAL, msg);
    }
    int device = 0;
    if (hipError_t e = hipGetDevice(&device); e != hipSuccess) return hip_fail(e, "hipGetDevice");
    cmlbm_lattice* h = new (std::nothrow) cmlbm_lattice();
    if (!h) return fail(CMLBM_ENOMEM, "host allocation failed");
    h->device = device;
    cm::LaunchArgs& a = h->a;
    a.g.nx = d->nx;
    a.g.ny = d->ny;
    a.g.nz = d->nz;
    a.g.N = N;
    {
        a.g.rowloop = (d->tuning & 4u) ? 1 : 0;
        a.g.lanegather = (d->tuning & 32u) ? 1 : 0;
        a.g.pairs_off = (d->tuning & 64u) ? 1 : 0;
        a.g.one_launch = (d->tuning & 128u) ? 1 : 0;
        const unsigned order = (d->tuning >> 3) & 3u;
        a.g.xcd = order == 1u ? 0 : (order == 2u ? 1 : (order == 3u ? kXcdRun : default_xcd_order(d->lattice, d->storage, d->nx, a.g.rowloop != 0, (d->walls & 1u) != 0,
                                                                                !a.g.lanegather && !a.g.pairs_off)));
        a.xcd_default = order == 0u ? 1 : 0;
        a.g.aa = inplace ? 1 : 0;
        a.g.ybase = 0;
        a.g.ystride = 1;
        a.g.yrows = d->ny;
    }
    a.lattice = d->lattice;
    a.storage = d->storage;
    a.walls = (int)(d->walls & 1u);
    a.rho0 = d->rho0;
    a.omega_shear = a.omega_bulk = 1.0;
    for (int k = 0; k < 3; ++k) a.omega3[k] = 1.0;
    a.omega4[0] = a.omega4[1] = 1.0;
    a.omega5 = a.omega6 = 1.0;
    a.cs_smag = 0.0;
    a.flags = 0;
    for (int k = 0; k < 3; ++k) {
        a.force[k] = 0.0;
        a.wall_u_lo[k] = d->wall_u_lo[k];
        a.wall_u_hi[k] = d->wall_u_hi[k];
    }
    a.force_field = nullptr;
    a.stream = hip_stream;
    a.stress_prev = nullptr;
    a.stress_next = nullptr;
    h->stress[0] = h->stress[1] = nullptr;
    h->stress_bytes = 0;
    h->buf[0] = buf_a;
    h->buf[1] = buf_b;
    h->cur = 0;
    h->bytes_each = bytes_each;
    h->nparts = cm::reduce_partials(a.g);
    hipError_t e = hipMalloc((void**)&h->scratch, sizeof(double) * (8 * h->nparts + 8));
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipMalloc(reduction scratch)");
    }
    *out = h;
    return CMLBM_OK;
}

cmlbm_status cmlbm_destroy(cmlbm_handle h) {
    if (!h) return CMLBM_OK;
    hipError_t e = hipSuccess;
    if (h->scratch) {
        // the scratch may still be in use by work queued on the stream
        e = hipStreamSynchronize((hipStream_t)h->a.stream);
        hipError_t e2 = hipFree(h->scratch);
        if (e == hipSuccess) e = e2;
    }
    delete h;
    return e == hipSuccess ? CMLBM_OK : hip_fail(e, "cmlbm_destroy");
}

cmlbm_status cmlbm_set_stream(cmlbm_handle h, void* hip_stream) {
    if (cmlbm_status s = check_handle(h)) return s;
    h->a.stream = hip_stream;
    return CMLBM_OK;
}

cmlbm_status cmlbm_set_relaxation(cmlbm_handle h, const cmlbm_relax* r) {
    // the arguments are validated before the handle so that the checks can be
    // exercised without a device
    if (!r) return fail(CMLBM_EINVAL, "relax must be non-null");
    const double rates[] = {r->omega_shear, r->omega_bulk, r->omega3[0], r->omega3[1], r->omega3[2],
                            r->omega4[0],   r->omega4[1],  r->omega5,    r->omega6};
    for (double w : rates)
        if (!rate_ok(w)) return fail(CMLBM_EINVAL, "relaxation rates must lie in (0, 2)");
    if (!(std::isfinite(r->cs_smag) && r->cs_smag >= 0.0)) return fail(CMLBM_EINVAL, "cs_smag must be finite and >= 0");
    if ((r->flags & ~7u) || r->reserved) return fail(CMLBM_EINVAL, "flags: only bits 0-2 are defined; reserved must be 0");
    if (cmlbm_status s = check_handle(h)) return s;
    if (r->flags & CMLBM_SGS_FORCE) {
        if (h->a.walls) return fail(CMLBM_EINVAL, "the sub-grid force needs a periodic lattice");
        if (h->a.g.aa) return fail(CMLBM_EINVAL, "the sub-grid force needs two-buffer streaming");
    }
    cm::LaunchArgs& a = h->a;
    a.omega_shear = r->omega_shear;
    a.omega_bulk = r->omega_bulk;
    for (int k = 0; k < 3; ++k) a.omega3[k] = r->omega3[k];
    a.omega4[0] = r->omega4[0];
    a.omega4[1] = r->omega4[1];
    a.omega5 = r->omega5;
    a.omega6 = r->omega6;
    a.cs_smag = r->cs_smag;
    a.flags = r->flags;
    return CMLBM_OK;
}

cmlbm_status cmlbm_set_force(cmlbm_handle h, const double uniform[3], const void* field) {
    if (cmlbm_status s = check_handle(h)) return s;
    for (int k = 0; k < 3; ++k) {
        const double v = uniform ? uniform[k] : 0.0;
        if (!std::isfinite(v)) return fail(CMLBM_EINVAL, "uniform force must be finite");
        h->a.force[k] = v;
    }
    h->a.force_field = field;
    return CMLBM_OK;
}

cmlbm_status cmlbm_init_equilibrium(cmlbm_handle h, const void* rho, const void* u, cmlbm_dtype dt) {
    if (cmlbm_status s = check_handle(h)) return s;
    if (cmlbm_status s = check_dtype(dt)) return s;
    if (!u) return fail(CMLBM_EINVAL, "u must be non-null");
    h->cur = 0;
    if (h->a.g.aa) h->a.g.aa = 1;   // in place: a new state is in the even arrangement
    hipError_t e = reset_stress(h);
    if (e == hipSuccess)
        e = h->a.lattice ? cm2::launch_init_equilibrium(h->a, h->buf[0], rho, u, (int)dt)
                         : cm::launch_init_equilibrium(h->a, h->buf[0], rho, u, (int)dt);
    return e == hipSuccess ? CMLBM_OK : hip_fail(e, "init_equilibrium");
}

cmlbm_status cmlbm_step(cmlbm_handle h, int64_t nsteps) {
    if (cmlbm_status s = check_handle(h)) return s;
    if (nsteps < 0) return fail(CMLBM_EINVAL, "nsteps must be >= 0");
    if (cmlbm_status s = check_sgs_ready(h)) return s;
    if (h->a.g.aa) {
        for (int64_t n = 0; n < nsteps; ++n) {
            hipError_t e = cm::launch_step_inplace(h->a, h->buf[0]);
            if (e != hipSuccess) return hip_fail(e, "step");
            h->a.g.aa = 3 - h->a.g.aa;
        }
        return CMLBM_OK;
    }
    for (int64_t n = 0; n < nsteps; ++n) {
        bind_stress(h);
        hipError_t e = h->a.lattice ? cm2::launch_step(h->a, h->buf[h->cur], h->buf[h->cur ^ 1])
                                    : cm::launch_step(h->a, h->buf[h->cur], h->buf[h->cur ^ 1]);
        if (e != hipSuccess) return hip_fail(e, "step");
        h->cur ^= 1;
    }
    return CMLBM_OK;
}

cmlbm_status cmlbm_step_from(cmlbm_handle h, const void* src, void* dst) {
    if (cmlbm_status s = check_handle(h)) return s;
    if (!src || !dst || src == dst) return fail(CMLBM_EINVAL, "src and dst must be distinct non-null buffers");
    if (h->a.flags & CMLBM_SGS_FORCE)
        return fail(CMLBM_EINVAL, "step_from does not carry the sub-grid stress; use cmlbm_step");
    if (h->a.g.aa) return fail(CMLBM_EINVAL, "step_from needs two-buffer streaming");
    hipError_t e = h->a.lattice ? cm2::launch_step(h->a, src, dst) : cm::launch_step(h->a, src, dst);
    return e == hipSuccess ? CMLBM_OK : hip_fail(e, "step_from");
}

cmlbm_status cmlbm_state_buffer(cmlbm_handle h, void** buf, size_t* bytes) {
    if (cmlbm_status s = check_handle(h)) return s;
    if (!buf) return fail(CMLBM_EINVAL, "buf must be non-null");
    *buf = h->buf[h->cur];
    if (bytes) *bytes = (size_t)lattice_q(h->a.lattice) * (size_t)h->a.g.N * elem_size(h->a.storage);
    return CMLBM_OK;
}

cmlbm_status cmlbm_read_moments(cmlbm_handle h, void* rho, void* u, cmlbm_dtype dt) {
    if (cmlbm_status s = check_handle(h)) return s;
    if (cmlbm_status s = check_dtype(dt)) return s;
    if (!rho || !u) return fail(CMLBM_EINVAL, "rho and u must be non-null");
    if (cmlbm_status s = check_sgs_ready(h)) return s;
    bind_stress(h);
    hipError_t e = h->a.lattice ? cm2::launch_read(h->a, h->buf[h->cur], rho, u, (int)dt, 1)
                                : cm::launch_read(h->a, h->buf[h->cur], rho, u, (int)dt, 1);
    return e == hipSuccess ? CMLBM_OK : hip_fail(e, "read_moments");
}

cmlbm_status cmlbm_get_populations(cmlbm_handle h, void* f, cmlbm_dtype dt) {
    if (cmlbm_status s = check_handle(h)) return s;
    if (cmlbm_status s = check_dtype(dt)) return s;
    if (!f) return fail(CMLBM_EINVAL, "f must be non-null");
    hipError_t e = h->a.lattice ? cm2::launch_read(h->a, h->buf[h->cur], f, nullptr, (int)dt, 0)
                                : cm::launch_read(h->a, h->buf[h->cur], f, nullptr, (int)dt, 0);
    return e == hipSuccess ? CMLBM_OK : hip_fail(e, "get_populations");
}

cmlbm_status cmlbm_set_populations(cmlbm_handle h, const void* f, cmlbm_dtype dt) {
    if (cmlbm_status s = check_handle(h)) return s;
    if (cmlbm_status s = check_dtype(dt)) return s;
    if (!f) return fail(CMLBM_EINVAL, "f must be non-null");
    if (h->a.g.aa) h->a.g.aa = 1;   // in place: set in the even arrangement
    hipError_t e = reset_stress(h);
    if (e == hipSuccess)
        e = h->a.lattice ? cm2::launch_set_populations(h->a, h->buf[h->cur], f, (int)dt)
                         : cm::launch_set_populations(h->a, h->buf[h->cur], f, (int)dt);
    return e == hipSuccess ? CMLBM_OK : hip_fail(e, "set_populations");
}

cmlbm_status cmlbm_reduce(cmlbm_handle h, double out[8]) {
    if (cmlbm_status s = check_handle(h)) return s;
    if (!out) return fail(CMLBM_EINVAL, "out must be non-null");
    if (cmlbm_status s = check_sgs_ready(h)) return s;
    bind_stress(h);
    double* res = h->scratch + 8 * h->nparts;
    hipError_t e = h->a.lattice ? cm2::launch_reduce(h->a, h->buf[h->cur], h->scratch, res)
                                : cm::launch_reduce(h->a, h->buf[h->cur], h->scratch, res);
    if (e == hipSuccess) e = hipMemcpyAsync(out, res, 8 * sizeof(double), hipMemcpyDeviceToHost, (hipStream_t)h->a.stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)h->a.stream);
    if (e != hipSuccess) return hip_fail(e, "reduce");
    if (out[5] > 0) {
        char msg[96];
        std::snprintf(msg, sizeof msg, "%.0f cells with non-finite rho or u", out[5]);
        return fail(CMLBM_ENONFINITE, msg);
    }
    return CMLBM_OK;
}

cmlbm_status cmlbm_reduce_noalloc(cmlbm_handle h, double* out) {
    if (cmlbm_status s = check_handle(h)) return s;
    if (!out) return fail(CMLBM_EINVAL, "out must be a non-null device array of 8 doubles");
    if (cmlbm_status s = check_sgs_ready(h)) return s;
    double* scratch = nullptr;
    hipError_t e = cm::static_reduce_scratch(h->device, &scratch);
    if (e != hipSuccess) return hip_fail(e, "reduce_noalloc: address of the static scratch");
    // the partial kernel launches at most kStaticReduceBlocks workgroups, so
    // every lattice fits; the check guards the array's size against changes
    const size_t nparts = std::min(h->nparts, cm::kStaticReduceBlocks);
    if (nparts > cm::kStaticReduceBlocks) return fail(CMLBM_EINVAL, "reduce_noalloc: partials exceed the static scratch");
    bind_stress(h);
    // partials in the static scratch, the final combination straight into out
    e = h->a.lattice ? cm2::launch_reduce(h->a, h->buf[h->cur], scratch, out, cm::kStaticReduceBlocks)
                     : cm::launch_reduce(h->a, h->buf[h->cur], scratch, out, cm::kStaticReduceBlocks);
    return e == hipSuccess ? CMLBM_OK : hip_fail(e, "reduce_noalloc");
}

static cmlbm_status adjoint_ok(cmlbm_handle h) {
    if (h->a.lattice != CMLBM_D3Q27) return fail(CMLBM_EINVAL, "adjoint supports the D3Q27 lattice only");
    if (h->a.g.aa) return fail(CMLBM_EINVAL, "adjoint needs two-buffer streaming");
    if (h->a.flags & CMLBM_SGS_FORCE) return fail(CMLBM_EINVAL, "adjoint does not support the sub-grid stress as a force");
    return CMLBM_OK;
}

cmlbm_status cmlbm_adjoint_step(cmlbm_handle h, const void* state, const void* lam_in, void* lam_out, void* grad_F) {
    if (cmlbm_status s = check_handle(h)) return s;
    if (cmlbm_status s = adjoint_ok(h)) return s;
    if (!state || !lam_in || !lam_out || !grad_F || lam_in == lam_out)
        return fail(CMLBM_EINVAL, "state, lam_in, lam_out, grad_F must be non-null and lam_in != lam_out");
    hipError_t e = cm::launch_adjoint(h->a, state, lam_in, lam_out, grad_F);
    return e == hipSuccess ? CMLBM_OK : hip_fail(e, "adjoint_step");
}

cmlbm_status cmlbm_energy_seed(cmlbm_handle h, const void* state, void* lam_out, void* grad_F) {
    if (cmlbm_status s = check_handle(h)) return s;
    if (cmlbm_status s = adjoint_ok(h)) return s;
    if (!state || !lam_out || !grad_F) return fail(CMLBM_EINVAL, "state, lam_out, grad_F must be non-null");
    hipError_t e = cm::launch_energy_seed(h->a, state, lam_out, grad_F);
    return e == hipSuccess ? CMLBM_OK : hip_fail(e, "energy_seed");
}

cmlbm_status cmlbm_set_sgs_buffers(cmlbm_handle h, void* stress_a, void* stress_b, size_t bytes_each) {
    if (cmlbm_status s = check_handle(h)) return s;
    if (h->a.g.aa) return fail(CMLBM_EINVAL, "the sub-grid force needs two-buffer streaming");
    if (!stress_a || !stress_b || stress_a == stress_b)
        return fail(CMLBM_EINVAL, "two distinct non-null stress buffers are required");
    const size_t es = h->a.storage == CMLBM_F64 ? 8 : 4;
    const size_t planes = h->a.lattice == CMLBM_D2Q9 ? 3 : 6;
    const size_t need = planes * (size_t)h->a.g.N * es;
    if (bytes_each < need) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "stress buffers too small: %zu bytes given, %zu needed", bytes_each, need);
        return fail(CMLBM_EINVAL, msg);
    }
    h->stress[0] = stress_a;
    h->stress[1] = stress_b;
    h->stress_bytes = need;
    hipError_t e = reset_stress(h);
    return e == hipSuccess ? CMLBM_OK : hip_fail(e, "set_sgs_buffers");
}

cmlbm_status cmlbm_copy(const void* src, void* dst, size_t bytes, void* hip_stream) {
    if (!src || !dst || src == dst) return fail(CMLBM_EINVAL, "src and dst must be distinct non-null buffers");
    if (bytes % 16 || ((uintptr_t)src % 16) || ((uintptr_t)dst % 16))
        return fail(CMLBM_EINVAL, "bytes and both addresses must be multiples of 16");
    hipError_t e = cm::launch_copy(src, dst, bytes, hip_stream);
    return e == hipSuccess ? CMLBM_OK : hip_fail(e, "copy");
}

}  // extern "C"
