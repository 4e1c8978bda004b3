#!/usr/bin/env python3
"""Throughput of the D3Q27 cascaded central-moment LES step on one MI355X.

Workload (the headline line): 256^3 periodic forced isotropic turbulence,
FP32 populations, Smagorinsky C_s = 0.12, omega_0 = 1.95, static solenoidal
band-limited forcing (|k| in [1, 2], rms 1e-4), initial solenoidal Gaussian
velocity with E(k) ~ k^4 exp(-2 (k/k0)^2), k0 = 4, per-component rms 0.03.
Inputs are seeded and synthetic and resident in HBM before timing starts.
One step = one launch of the fused pull-stream + collide kernel over all
cells. Prints one JSON line (MLUPS, roofline, oracle CPU baseline) and, unless
--extras none, the relaxation variants (the Sec. 12-14 operators on the same
workload), the adjoint (128^3), the paper's D2Q9 lattice (8192^2), in-place
streaming (256^3 and 1024^3), a walled channel (256^3), the two small
cache-resident configurations (32^3 FP64 Taylor-Green, 64 x 64 x 128 channel)
and the reduced-precision (512^3) modes in the same line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ["paper_1202_6074_amd/csrc/cm_math.hpp", "paper_1202_6074_amd/csrc/kernels.hip",
                  "paper_1202_6074_amd/csrc/store.hpp", "paper_1202_6074_amd/csrc/cm_math2d.hpp",
                  "paper_1202_6074_amd/csrc/kernels2d.hip"]
EXTRAS = ("variants", "adjoint", "d2q9", "inplace", "channel", "precision", "small")


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_entry(kernel_key):
    """The committed rocprofv3 counter summary of a kernel (HBM bytes per launch,
    cells per launch, bytes per cell), or None when it was taken on other
    kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    ent = data.get(kernel_key)
    if not ent or ent.get("source_hash") != kernel_hash():
        return None
    return ent


def measured_traffic(kernel_key):
    """HBM bytes of one launch (and the cells it updates) from committed
    rocprofv3 counter summaries, or None."""
    ent = traffic_entry(kernel_key)
    if not ent:
        return None
    return {"bytes_per_launch": ent.get("bytes_per_launch"), "cells_per_launch": ent.get("cells"),
            "bytes_per_cell": ent.get("bytes_per_cell")}


def timed_steps(lat, steps, warmup, segments=None):
    """Seconds for `steps` steps after `warmup` untimed ones, HIP events on the
    lattice's stream. With a list `segments`, the timed region is also cut into
    5 equal parts by events recorded in between (no synchronisation), whose
    per-step times are appended to it."""
    import torch
    lat.step(warmup)
    torch.cuda.synchronize()
    stream = lat.stream
    nseg = 5 if segments is not None and steps >= 5 else 1
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nseg + 1)]
    ev[0].record(stream)
    done = 0
    for k in range(nseg):
        n = (steps - done) // (nseg - k)
        lat.step(n)
        done += n
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    if nseg > 1:
        done = 0
        for k in range(nseg):
            n = (steps - done) // (nseg - k)
            done += n
            segments.append(ev[k].elapsed_time(ev[k + 1]) / 1e3 / n)
    return ev[0].elapsed_time(ev[nseg]) / 1e3   # seconds


def copy_bandwidth(nbytes=4 << 30, reps=20, min_seconds=0.5):
    """Achievable HBM bandwidth of a plain streaming copy kernel (read + write bytes / time).

    The copy runs back to back for at least `min_seconds` before the `reps`
    timed copies: after the GPU has been idle (e.g. while inputs are generated
    on the host) the first ~10 ms of kernels run up to 15 % slower, so this
    also brings the GPU to its sustained state before the headline steps."""
    import torch

    from paper_1202_6074_amd import _lib
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    st = torch.cuda.current_stream()
    t0 = time.time()
    while time.time() - t0 < min_seconds:
        for _ in range(20):
            _lib.cmlbm_copy(a.data_ptr(), b.data_ptr(), nbytes, st.cuda_stream)
        torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        _lib.cmlbm_copy(a.data_ptr(), b.data_ptr(), nbytes, st.cuda_stream)
    e1.record(st)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / t / 1e9


def les_lattice(n, storage, device="cuda", in_place=False):
    import torch

    import synth
    from paper_1202_6074_amd.lattice import Lattice
    shape = (n, n, n)
    t = time.time()
    u = synth.turbulence_velocity(shape, k0=4.0, urms=0.03)
    F = synth.band_forcing(shape, frms=1e-4)
    log(f"inputs {n}^3 generated in {time.time() - t:.1f} s")
    lat = Lattice(shape, storage=storage, in_place=in_place)
    lat.set_relaxation(1.95, cs_smag=0.12)
    lat.set_force((0, 0, 0), torch.tensor(F, device=device, dtype=lat.dtype))
    lat.init_equilibrium(torch.tensor(u, device=device, dtype=torch.float32))
    torch.cuda.synchronize()
    del u, F
    return lat


D2Q9_N = 8192


def d2q9_lattice(n, storage, device="cuda"):
    """The paper's own lattice: 2D forced turbulence, n^2 periodic, LES."""
    import torch

    import synth
    from paper_1202_6074_amd.lattice import Lattice
    u = synth.turbulence_velocity_2d((n, n), k0=8.0, urms=0.03)
    F = synth.kolmogorov_force_2d((n, n), kf=4, amp=1e-5)
    lat = Lattice((n, n), storage=storage, lattice="d2q9")
    lat.set_relaxation(1.95, cs_smag=0.12)
    lat.set_force((0, 0, 0), torch.tensor(F, device=device, dtype=lat.dtype))
    lat.init_equilibrium(torch.tensor(u, device=device, dtype=torch.float32))
    torch.cuda.synchronize()
    del u, F
    return lat


def d2q9_section(steps, warmup):
    """D2Q9 step kernel (FP32 LES, force field) at 8192^2, MLUPS and bytes."""
    import torch
    n = D2Q9_N
    lat = d2q9_lattice(n, "f32")
    dt = timed_steps(lat, steps, warmup)
    red = lat.reduce(raise_nonfinite=False)
    bpc = 9 * 4 * 2 + 8
    gbs = bpc * n * n / (dt / steps) / 1e9
    out = {"workload": f"D2Q9 cascaded LES, FP32, {n}^2 periodic 2D turbulence (Cs=0.12, omega0=1.95, "
                       "Kolmogorov forcing k=4 amplitude 1e-5, k0=8 rms 0.03)",
           "kernel": f"k2_step<f32,periodic,les,force_field>@{n}^2", "steps": steps,
           "mlups": round(n * n * steps / dt / 1e6, 1), "bytes_per_cell": bpc, "gbs": round(gbs, 1),
           "frac_of_peak": round(gbs / PEAK_HBM_GBS, 4),
           "traffic": measured_traffic(f"k2_step<f32,periodic,les,force_field>@{n}^2"),
           "ke": red["ke"], "nonfinite": red["nonfinite"]}
    del lat
    torch.cuda.empty_cache()
    return out


def inplace_section(steps, warmup):
    """In-place streaming (one population buffer): the headline workload, and
    1024^3 LES lattices in FP32 and FP16-shifted storage (116 GB and 58 GB of
    populations instead of twice that)."""
    import torch

    from paper_1202_6074_amd.lattice import Lattice
    out = {}
    lat = les_lattice(256, "f32", in_place=True)
    dt = timed_steps(lat, steps, warmup)
    N = 256 ** 3
    out["256^3_f32"] = {"mlups": round(N * steps / dt / 1e6, 1), "gbs": round(228 * N / (dt / steps) / 1e9, 1),
                        "buffers": 1, "kernel": "k_step_inplace<f32,periodic,les,force_field> (even/odd)",
                        "traffic": {"even": measured_traffic("k_step_inplace<f32,periodic,les,force_field,even>@256^3"),
                                    "odd": measured_traffic("k_step_inplace<f32,periodic,les,force_field,odd>@256^3")}}
    lat.close()
    del lat
    torch.cuda.empty_cache()
    n = 1024
    x = torch.arange(n, device="cuda", dtype=torch.float32) * (2 * 3.141592653589793 / n)
    for storage, elem in (("f32", 4), ("f16s", 2)):
        lat = Lattice((n, n, n), storage=storage, in_place=True)
        lat.set_relaxation(1.95, cs_smag=0.12)
        F = torch.empty((3, n, n, n), device="cuda", dtype=torch.float32)
        F[0] = 1e-5 * torch.sin(x)[None, :, None]
        F[1] = 1e-5 * torch.sin(x)[:, None, None]
        F[2] = 1e-5 * torch.sin(x)[None, None, :]
        lat.set_force((0, 0, 0), F)
        u = torch.empty((3, n, n, n), device="cuda", dtype=torch.float32)
        u[0] = 0.03 * torch.sin(x)[None, None, :] * torch.cos(x)[None, :, None] * torch.cos(x)[:, None, None]
        u[1] = -0.03 * torch.cos(x)[None, None, :] * torch.sin(x)[None, :, None] * torch.cos(x)[:, None, None]
        u[2] = 0.0
        lat.init_equilibrium(u)
        del u
        torch.cuda.synchronize()
        s_big = max(10, steps // 20)
        dt = timed_steps(lat, s_big, min(warmup, 20))
        red = lat.reduce(raise_nonfinite=False)
        N = n ** 3
        bpc = 27 * elem * 2 + 12
        ent = {"mlups": round(N * s_big / dt / 1e6, 1), "bytes_per_cell": bpc,
               "gbs": round(bpc * N / (dt / s_big) / 1e9, 1), "steps": s_big,
               "population_bytes": lat.buf[0].numel() * lat.buf[0].element_size(), "nonfinite": red["nonfinite"]}
        if storage == "f32":
            ent["traffic"] = {"even": measured_traffic("k_step_inplace<f32,periodic,les,force_field,even>@1024^3"),
                              "odd": measured_traffic("k_step_inplace<f32,periodic,les,force_field,odd>@1024^3")}
        out[f"1024^3_{storage}"] = ent
        lat.close()
        del lat, F
        torch.cuda.empty_cache()
    out["note_1024"] = ("1024^3 lattices with a Taylor-Green-type initial field and force built on the GPU "
                        "(the timing does not depend on the values); one buffer of populations (116 GB FP32, "
                        "58 GB FP16) instead of two")
    return out


def channel_section(steps, warmup):
    """Walled channel (halfway bounce-back at y = -1/2 and 255.5, one wall moving),
    256^3 FP32, LES, uniform body force: the wall path's throughput."""
    import torch

    from paper_1202_6074_amd.lattice import Lattice
    n = 256
    lat = Lattice((n, n, n), storage="f32", walls=True, wall_u_hi=(0.02, 0.0, 0.0))
    lat.set_relaxation(1.95, cs_smag=0.12)
    lat.set_force((1e-6, 0.0, 0.0))
    lat.init_equilibrium(torch.zeros((3, n, n, n), device="cuda"))
    dt = timed_steps(lat, steps, warmup)
    N = n ** 3
    out = {"workload": "D3Q27 cascaded LES, FP32, 256^3 channel (walls at y = -1/2, 255.5; upper wall "
                       "U = 0.02; F_x = 1e-6; Cs = 0.12, omega0 = 1.95)",
           "mlups": round(N * steps / dt / 1e6, 1), "bytes_per_cell": 216,
           "gbs": round(216 * N / (dt / steps) / 1e9, 1),
           "kernels": {"interior_rows": "k_step<f32,interior_rows,les,uniform_force>@256^3_channel",
                       "wall_rows": "k_step<f32,wall_rows,les,uniform_force>@256^3_channel"},
           "traffic": {"interior_rows": measured_traffic("k_step<f32,interior_rows,les,uniform_force>@256^3_channel"),
                       "wall_rows": measured_traffic("k_step<f32,wall_rows,les,uniform_force>@256^3_channel")},
           "note": "uniform force: 27 x 4 x 2 bytes per cell; wall rows run a kernel of their own"}
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return out


def timed_graph(lat, reinit, steps, per_graph, warmup=0):
    """Seconds for `steps` steps replayed from a HIP graph of `per_graph`
    captured steps (Lattice.capture_steps), HIP events on the lattice's stream.
    One untimed replay first (the graph's first launch uploads it), then
    reinit() and `warmup` eager steps, so that the timed replays start from
    the same state as the eager measurement."""
    import torch
    g = lat.capture_steps(per_graph)
    g.replay()
    torch.cuda.synchronize()
    reinit()
    lat.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    g.replay(steps // per_graph)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def small_section():
    """The two small configurations, MLUPS only: 32^3 FP64 Taylor-Green vortex
    (u0 = 0.02, omega = 1.6, uniform F = (1e-5, 0, 0), 200 steps) and the
    64 x 64 x 128 FP32 channel (walls at y = -1/2 and 63.5, F_x = 1e-6,
    omega = 1.2; 2000 of its 20000 steps, from rest). Their 14 MB and 113 MB
    of populations sit in the 256 MB Infinity Cache and a step lasts a few
    microseconds, so launch and cache latency set these rates, not HBM."""
    import torch

    import synth
    from paper_1202_6074_amd.lattice import Lattice
    out = {}
    n = 32
    lat = Lattice((n, n, n), storage="f64")
    lat.set_relaxation(1.6)
    lat.set_force((1e-5, 0.0, 0.0))
    rho, u = synth.taylor_green_3d((n, n, n), u0=0.02)
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    lat.step(20)
    torch.cuda.synchronize()
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    dt = timed_steps(lat, 200, 0)
    ke = lat.reduce()["ke"]
    out["tgv_32^3_f64"] = {"mlups": round(n ** 3 * 200 / dt / 1e6, 1), "us_per_step": round(dt / 200 * 1e6, 2),
                           "steps": 200, "ke": ke}
    dt = timed_graph(lat, lambda: lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda")),
                     200, 100)
    out["tgv_32^3_f64"]["graph"] = {"mlups": round(n ** 3 * 200 / dt / 1e6, 1), "us_per_step": round(dt / 200 * 1e6, 2),
                                    "steps_per_graph": 100, "state_equal_to_eager": lat.reduce()["ke"] == ke}
    lat.close()
    nx, ny, nz = 64, 64, 128
    lat = Lattice((nx, ny, nz), storage="f32", walls=True)
    lat.set_relaxation(1.2)
    lat.set_force((1e-6, 0.0, 0.0))
    lat.init_equilibrium(torch.zeros((3, nz, ny, nx), device="cuda"))
    dt = timed_steps(lat, 2000, 100)
    N = nx * ny * nz
    ke = lat.reduce()["ke"]
    out["channel_64x64x128_f32"] = {"mlups": round(N * 2000 / dt / 1e6, 1), "us_per_step": round(dt / 2000 * 1e6, 2),
                                    "steps": 2000}
    dt = timed_graph(lat, lambda: lat.init_equilibrium(torch.zeros((3, nz, ny, nx), device="cuda")), 2000, 200, 100)
    out["channel_64x64x128_f32"]["graph"] = {"mlups": round(N * 2000 / dt / 1e6, 1),
                                             "us_per_step": round(dt / 2000 * 1e6, 2), "steps_per_graph": 200,
                                             "state_equal_to_eager": lat.reduce()["ke"] == ke}
    lat.close()
    out["note"] = ("cache-resident, launch-bound sizes: MLUPS only (no HBM roofline); 'graph': the same steps "
                   "replayed from a HIP graph (Lattice.capture_steps)")
    return out


def bytes_per_cell(storage_elem, force_bytes):
    return 27 * storage_elem * 2 + force_bytes


def cpu_baseline():
    """The FP64 NumPy oracle on the host, on a bounded sample of the same workload."""
    import numpy as np

    import synth
    from oracle.lattice import Relax
    from oracle.sim import OracleSim
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        threads = 1
    n, steps = 64, 60
    shape = (n, n, n)
    u = synth.turbulence_velocity(shape, k0=4.0, urms=0.03)
    F = synth.band_forcing(shape, frms=1e-4)
    sim = OracleSim(shape, Relax(omega_shear=1.95, cs_smag=0.12), force=F.reshape(3, -1))
    sim.init_equilibrium(np.ones(shape), u)
    sim.step(1)
    t = time.time()
    sim.step(steps)
    dt = time.time() - t
    out = {"value": round(n ** 3 * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": int(threads), "kind": "oracle",
           "sample": f"{n}^3 cells x {steps} steps of the same LES workload (FP64 NumPy oracle, "
                     f"{dt:.1f} s; BLAS threads {threads}, element-wise NumPy single-threaded)"}
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(line.split(":", 1)[1].strip() for line in fh if line.startswith("model name"))
    except Exception:
        pass
    out["host"] = {"nproc": os.cpu_count(), "cpu": cpu}
    # the 32^3 FP64 Taylor-Green configuration (200 steps) in full
    rho, u = synth.taylor_green_3d((32, 32, 32), u0=0.02)
    sim = OracleSim((32, 32, 32), Relax(omega_shear=1.6), force=(1e-5, 0.0, 0.0))
    sim.init_equilibrium(rho, u)
    t = time.time()
    sim.step(200)
    dt2 = time.time() - t
    out["taylor_green_32^3_200_steps"] = {"seconds": round(dt2, 2), "mlups": round(32 ** 3 * 200 / dt2 / 1e6, 4)}
    return out


def _adjoint_lattice(n, storage):
    """Periodic n^3 lattice at rest, omega = 1.6, no force bound yet; returns it and
    a copy of its initial state."""
    import torch

    from paper_1202_6074_amd.lattice import Lattice
    lat = Lattice((n, n, n), storage=storage)
    lat.set_relaxation(1.6)
    lat.set_force((0, 0, 0), torch.zeros((3, n, n, n), device="cuda", dtype=lat.dtype))
    lat.init_equilibrium(torch.zeros((3, n, n, n), device="cuda"))
    return lat, lat.state_buffer().clone()


def _adjoint_kernel_seconds(lat, state, n, reps=200):
    """Average time of one adjoint-step launch on resident buffers (HIP events)."""
    import torch
    lam = lat.lam_buffer().zero_()
    lam2 = torch.zeros_like(lam)
    g = torch.zeros((3, n, n, n), device="cuda", dtype=lat.dtype)
    for _ in range(5):
        lat.adjoint_step(state, lam, lam2, g)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    for _ in range(reps):
        lat.adjoint_step(state, lam, lam2, g)
        lam, lam2 = lam2, lam
    e1.record(lat.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def _timed_passes(lat, F, f0, steps, K):
    """(E, dE/dF, forward seconds, backward seconds), host wall clock around
    synchronised passes."""
    import torch

    from paper_1202_6074_amd.adjoint import _backward, _forward
    torch.cuda.synchronize()
    t = time.time()
    E, ckpts, final = _forward(lat, F, f0, steps, K)
    torch.cuda.synchronize()
    t_fwd = time.time() - t
    t = time.time()
    gF = _backward(lat, F, ckpts, final, steps, K)
    torch.cuda.synchronize()
    t_bwd = time.time() - t
    del ckpts, final
    return E, gF, t_fwd, t_bwd


def adjoint_section(steps=500, K=50):
    """The adjoint workload (128^3 periodic FP32, smooth random force parameter,
    E = kinetic energy at step `steps`, checkpoints every K): rates, and the
    gradient's accuracy against central differences of E in FP64 storage and
    against the FP64 adjoint. Then the same at 256^3, where the working set is
    far larger than the Infinity Cache (HBM rates)."""
    import torch

    import synth
    n = 128
    shape = (n, n, n)
    N = n ** 3
    Fnp = synth.smooth_random_force(shape, sigma=4.0, frms=1e-5)
    F = torch.tensor(Fnp, device="cuda", dtype=torch.float32)
    lat, f0 = _adjoint_lattice(n, "f32")
    E, gF, t_fwd, t_bwd = _timed_passes(lat, F, f0, steps, K)
    t_adj = _adjoint_kernel_seconds(lat, f0, n)
    gnorm = float(gF.double().norm())
    torch.cuda.empty_cache()
    # every state kept (500 x 226 MB in HBM): no recomputation in the backward pass
    E_all, gF_all, t_fwd_all, t_bwd_all = _timed_passes(lat, F, f0, steps, steps)
    same = bool(E_all == E and torch.equal(gF_all, gF))
    del gF_all
    lat.close()
    del lat, f0
    torch.cuda.empty_cache()
    # accuracy: FP64 adjoint, and central differences of E in FP64 storage along
    # seeded smooth random directions (Richardson-extrapolated from h and 2h)
    lat64, f064 = _adjoint_lattice(n, "f64")
    F64 = F.double()
    E64, g64, _, _ = _timed_passes(lat64, F64, f064, steps, K)
    g32 = gF.double()
    h = 1e-2
    fd = []
    for k in range(4):
        v = torch.tensor(synth.smooth_random_force(shape, sigma=4.0, frms=1e-5, seed=1000 + k), device="cuda")
        e = {}
        for sgn in (-2, -1, 1, 2):
            lat64.set_force((0, 0, 0), F64 + sgn * h * v)
            lat64.state_buffer().copy_(f064)
            lat64.step(steps)
            e[sgn] = lat64.reduce()["ke"]
        d = (4 * (e[1] - e[-1]) / (2 * h) - (e[2] - e[-2]) / (4 * h)) / 3
        fd.append({"fd": d, "fp32_adjoint_rel_err": abs(float((g32 * v).sum()) - d) / abs(d),
                   "fp64_adjoint_rel_err": abs(float((g64 * v).sum()) - d) / abs(d)})
    acc = {"E_fp64": E64, "E_fp32_rel_err": abs(E - E64) / E64,
           "grad_fp32_vs_fp64_rel_l2": float((g32 - g64).norm() / g64.norm()),
           "directional_derivatives": fd,
           "note": "<dE/dF, v> along 4 seeded smooth random directions v (rms 1e-5) against central "
                   "differences of E from FP64-storage forward runs, steps h = 0.01 and 2h combined "
                   "(Richardson)"}
    lat64.close()
    del lat64, f064, g64, gF, g32
    torch.cuda.empty_cache()
    out = {"workload": f"adjoint {n}^3 FP32, E = kinetic energy at step {steps}, checkpoints every {K}",
           "E": E, "grad_norm": gnorm,
           "adjoint_kernel_mlups": round(N / t_adj / 1e6, 1),
           "adjoint_kernel_gbs": round(360 * N / t_adj / 1e9, 1),
           "adjoint_kernel": f"k_adjoint<f32,force_field>@{n}^3",
           "adjoint_kernel_traffic": measured_traffic(f"k_adjoint<f32,force_field>@{n}^3"),
           "forward_with_checkpoints_mlups": round(N * steps / t_fwd / 1e6, 1),
           "backward_end_to_end_mlups": round(N * steps / t_bwd / 1e6, 1),
           "keep_every_state": {"forward_mlups": round(N * steps / t_fwd_all / 1e6, 1),
                                "backward_mlups": round(N * steps / t_bwd_all / 1e6, 1),
                                "state_bytes": steps * 27 * N * 4,
                                "gradient_bitwise_equal_to_checkpointed": same},
           "accuracy": acc,
           "note": "backward = recompute + adjoint; host-timed wall clock. The 128^3 FP32 ping-pong "
                   "buffers (453 MB) partly fit the 256 MB Infinity Cache, so these rates are not pure HBM rates. "
                   "keep_every_state: the forward run keeps all 500 states and the backward runs the adjoint "
                   "steps only"}
    # HBM scale: 256^3 (1.8 GB per population buffer, 60 of them for K = 50)
    n2 = 256
    N2 = n2 ** 3
    F2 = torch.tensor(synth.smooth_random_force((n2, n2, n2), sigma=4.0, frms=1e-5), device="cuda",
                      dtype=torch.float32)
    lat, f0 = _adjoint_lattice(n2, "f32")
    E2, g2, t_fwd2, t_bwd2 = _timed_passes(lat, F2, f0, steps, K)
    t_adj2 = _adjoint_kernel_seconds(lat, f0, n2, reps=100)
    key2 = f"k_adjoint<f32,force_field>@{n2}^3"
    # the adjoint of the LES collision (Smagorinsky C_s = 0.12) on the flow the
    # forward pass left: same bytes, the eddy rate's reverse mode in registers
    st_end = lat.state_buffer().clone()
    lat.set_relaxation(1.6, cs_smag=0.12)
    t_les = _adjoint_kernel_seconds(lat, st_end, n2, reps=100)
    # and with the Sec. 12-13 operators as well (the paper's recommended LES collision)
    lat.set_relaxation(1.6, cs_smag=0.12, factorized=True, reduced_compressibility=True)
    t_var = _adjoint_kernel_seconds(lat, st_end, n2, reps=100)
    lat.set_relaxation(1.6)
    del st_end
    key_les = f"k_adjoint<f32,force_field,les>@{n2}^3"
    key_var = f"k_adjoint<f32,force_field,les,var>@{n2}^3"
    out[f"{n2}^3"] = {"E": E2, "grad_norm": float(g2.double().norm()),
                      "adjoint_kernel_mlups": round(N2 / t_adj2 / 1e6, 1),
                      "adjoint_kernel_gbs": round(360 * N2 / t_adj2 / 1e9, 1),
                      "adjoint_kernel_frac_of_peak": round(360 * N2 / t_adj2 / 1e9 / PEAK_HBM_GBS, 4),
                      "adjoint_kernel": key2, "adjoint_kernel_traffic": measured_traffic(key2),
                      "les_adjoint_kernel_mlups": round(N2 / t_les / 1e6, 1),
                      "les_adjoint_kernel_frac_of_peak": round(360 * N2 / t_les / 1e9 / PEAK_HBM_GBS, 4),
                      "les_adjoint_kernel": key_les, "les_adjoint_kernel_traffic": measured_traffic(key_les),
                      "les_var_adjoint_kernel_mlups": round(N2 / t_var / 1e6, 1),
                      "les_var_adjoint_kernel_frac_of_peak": round(360 * N2 / t_var / 1e9 / PEAK_HBM_GBS, 4),
                      "les_var_adjoint_kernel": key_var, "les_var_adjoint_kernel_traffic": measured_traffic(key_var),
                      "forward_with_checkpoints_mlups": round(N2 * steps / t_fwd2 / 1e6, 1),
                      "backward_end_to_end_mlups": round(N2 * steps / t_bwd2 / 1e6, 1),
                      "note": f"same workload at {n2}^3 ({steps} steps, checkpoints every {K}); "
                              "backward = recompute + adjoint, host-timed"}
    lat.close()
    del lat, f0, F2, g2
    torch.cuda.empty_cache()
    return out


def shell_spectrum_gpu(u):
    """Shell-summed kinetic-energy spectrum of a (3, n, n, n) field on the GPU (diagnostic)."""
    import torch
    n = u.shape[-1]
    hat = torch.fft.rfftn(u, dim=(1, 2, 3)) / n ** 3
    k1 = torch.fft.fftfreq(n, d=1.0 / n, device=u.device)
    kr = torch.fft.rfftfreq(n, d=1.0 / n, device=u.device)
    kk = torch.sqrt(k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + kr[None, None, :] ** 2)
    w = torch.where(kr == 0, 1.0, 2.0).to(u.dtype)
    if n % 2 == 0:
        w = torch.where(kr == n // 2, 1.0, w).to(u.dtype)
    e = 0.5 * (hat.real ** 2 + hat.imag ** 2).sum(0) * w[None, None, :]
    idx = torch.round(kk).long().reshape(-1)
    spec = torch.zeros(int(idx.max()) + 1, dtype=u.dtype, device=u.device)
    spec.index_add_(0, idx, e.reshape(-1))
    return spec


def precision_section(steps):
    """512^3 LES in FP16- and FP32-shifted storage (FP32 arithmetic) and FP64, MLUPS each,
    with the velocity error of the reduced-storage runs against the FP64 run."""
    import torch

    import synth
    from paper_1202_6074_amd.lattice import Lattice
    n = 512
    shape = (n, n, n)
    t = time.time()
    u = synth.turbulence_velocity(shape, k0=4.0, urms=0.03)
    F = synth.band_forcing(shape, frms=1e-4)
    log(f"512^3 inputs generated in {time.time() - t:.1f} s")
    u_dev = torch.tensor(u, device="cuda", dtype=torch.float32)
    F_dev = torch.tensor(F, device="cuda", dtype=torch.float64)
    del u, F
    res = {}
    u_ref = None
    N = n ** 3
    for storage, elem, fb in (("f64", 8, 24), ("f32s", 4, 12), ("f16s", 2, 12)):
        lat = Lattice(shape, storage=storage)
        lat.set_relaxation(1.95, cs_smag=0.12)
        lat.set_force((0, 0, 0), F_dev.to(lat.dtype))
        lat.init_equilibrium(u_dev)
        dt = timed_steps(lat, steps, 0)
        _, uu = lat.moments(torch.float64)
        red = lat.reduce(raise_nonfinite=False)
        key = f"k_step<{storage},periodic,les,force_field>@{n}^3"
        ent = {"kernel": key, "traffic": measured_traffic(key),
               "mlups": round(N * steps / dt / 1e6, 1), "bytes_per_cell": bytes_per_cell(elem, fb),
               "gbs": round(bytes_per_cell(elem, fb) * N * steps / dt / 1e9, 1), "ke": red["ke"],
               "nonfinite": red["nonfinite"]}
        spec = shell_spectrum_gpu(uu)
        if u_ref is None:
            u_ref, spec_ref = uu, spec
        else:
            d = uu - u_ref
            ent["u_err_rms_rel"] = float(d.pow(2).mean().sqrt() / u_ref.pow(2).mean().sqrt())
            ent["u_err_max"] = float(d.abs().max())
            ent["ke_rel_err"] = (red["ke"] - res["f64"]["ke"]) / res["f64"]["ke"]
            kmax = min(32, len(spec_ref) - 1)
            rel = (spec[1:kmax + 1] - spec_ref[1:kmax + 1]).abs() / spec_ref[1:kmax + 1]
            ent["spectrum_max_rel_err_k1_32"] = float(rel.max())
        res[storage] = ent
        log(f"precision {storage}: {ent}")
        del lat, uu
        torch.cuda.empty_cache()
    res["workload"] = (f"512^3 LES as the headline workload, {steps} timed steps from the initial state; "
                       "velocity, kinetic energy and shell spectrum (k = 1..32) errors vs the FP64 run")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip every extra section (same as --extras none)")
    ap.add_argument("--extras", default=",".join(EXTRAS),
                    help="comma-separated extra sections to run after the headline line: "
                         + ", ".join(EXTRAS) + " (or 'none')")
    ap.add_argument("--precision-steps", type=int, default=500)
    args = ap.parse_args()
    extras = set() if args.no_extras or args.extras == "none" else set(args.extras.split(","))
    unknown = extras - set(EXTRAS)
    if unknown:
        ap.error(f"unknown extra sections: {sorted(unknown)}")
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_1202_6074_amd import _lib
    _lib.load()

    n = 256
    N = n ** 3
    lat = les_lattice(n, "f32")
    # the copy kernel's bandwidth (reported below) is measured first: it also
    # ends the GPU's idle time while the inputs were generated on the host
    copy_gbs = copy_bandwidth()
    log(f"copy kernel: {copy_gbs:.0f} GB/s")
    log("warm-up and timed steps")
    seg = []
    dt = timed_steps(lat, args.steps, args.warmup, seg)
    red = lat.reduce(raise_nonfinite=False)
    ms = dt / args.steps * 1e3
    mlups = N * args.steps / dt / 1e6
    bpc = bytes_per_cell(4, 12)
    achieved = bpc * N / (dt / args.steps) / 1e9
    kernel_key = "k_step<f32,periodic,les,force_field>@256^3"
    tr_ent = traffic_entry(kernel_key)
    traffic = tr_ent.get("bytes_per_launch") if tr_ent else None
    line = {
        "metric": "MLUPS and % HBM roofline for D3Q27 cascaded LES step; adjoint MLUPS",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "D3Q27 cascaded LES, FP32, 256^3 periodic forced isotropic turbulence "
                               "(Cs=0.12, omega0=1.95, band forcing |k|=1..2 rms 1e-4, k0=4 rms 0.03)",
                   "cells": N, "global_batch": 1, "parallelism": "none (one GPU)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic, "kernel": kernel_key, "bytes_per_cell": bpc,
                     "traffic_bytes_per_cell": tr_ent.get("bytes_per_cell") if tr_ent else None,
                     "launches_per_step": 2, "cells_per_launch": N // 2,
                     "note": "one step = two launches of 128 z-planes each; achieved = algorithmic bytes / "
                             "time per step, the same as per launch"},
        "state_after": {"ke": red["ke"], "nonfinite": red["nonfinite"], "mass": red["mass"]},
        "timing": {"segments_ms_per_step": [round(t * 1e3, 4) for t in seg],
                   "median_segment_mlups": round(N / sorted(seg)[len(seg) // 2] / 1e6, 1) if seg else None,
                   "note": "the timed steps cut into 5 equal segments by events recorded between them"},
    }
    log(f"main: {mlups:.0f} MLUPS, {achieved:.0f} GB/s")
    line["roofline"]["copy_kernel_gbs"] = round(copy_gbs, 1)
    line["roofline"]["frac_of_copy"] = round(achieved / copy_gbs, 4)
    if "variants" in extras:
        # the paper's recommended operator for filtered flows: factorized attractors +
        # reduced compressibility (Secs. 12-13), same workload and buffers
        lat.set_relaxation(1.95, cs_smag=0.12, factorized=True, reduced_compressibility=True)
        dtv = timed_steps(lat, args.steps, args.warmup)
        key_v = "k_step<f32,periodic,les,force_field,var>@256^3"
        line["variants"] = {"factorized_reduced_compressibility": {
            "mlups": round(N * args.steps / dtv / 1e6, 1), "bytes_per_cell": bpc,
            "gbs": round(bpc * N / (dtv / args.steps) / 1e9, 1), "kernel": key_v,
            "traffic": measured_traffic(key_v),
            "note": "same 256^3 FP32 LES workload, continued from the headline run's state"}}
        log(f"variant RC+factorized: {N * args.steps / dtv / 1e6:.0f} MLUPS")
        # the complete Sec. 14 operator: the same, with the sub-grid stress as a force
        # (reads the previous stress field around each cell, writes this step's)
        lat.set_relaxation(1.95, cs_smag=0.12, factorized=True, reduced_compressibility=True, sgs_force=True)
        dts = timed_steps(lat, args.steps, args.warmup)
        bpc_s = bpc + 6 * 4 * 2
        red_s = lat.reduce(raise_nonfinite=False)
        key_s = "k_step<f32,periodic,sgs_force,force_field,var>@256^3"
        line["variants"]["sgs_force_factorized_reduced_compressibility"] = {
            "mlups": round(N * args.steps / dts / 1e6, 1), "bytes_per_cell": bpc_s,
            "gbs": round(bpc_s * N / (dts / args.steps) / 1e9, 1), "kernel": key_s,
            "traffic": measured_traffic(key_s), "nonfinite": red_s["nonfinite"],
            "note": "Sec. 14 coupling, same workload, continued from the previous state"}
        log(f"variant SGS force: {N * args.steps / dts / 1e6:.0f} MLUPS")
    del lat
    torch.cuda.empty_cache()
    if "adjoint" in extras:
        try:
            log("adjoint section")
            line["adjoint"] = adjoint_section()
        except Exception as e:  # report and keep the headline line
            line["adjoint"] = {"error": repr(e)}
    if "d2q9" in extras:
        try:
            log("d2q9 section")
            line["d2q9"] = d2q9_section(args.steps, args.warmup)
            log(f"d2q9: {line['d2q9']['mlups']:.0f} MLUPS, {line['d2q9']['gbs']:.0f} GB/s")
        except Exception as e:
            line["d2q9"] = {"error": repr(e)}
    if "inplace" in extras:
        try:
            log("in-place streaming section")
            line["inplace"] = inplace_section(args.steps, args.warmup)
        except Exception as e:
            line["inplace"] = {"error": repr(e)}
    if "channel" in extras:
        try:
            log("channel section")
            line["channel"] = channel_section(args.steps, args.warmup)
        except Exception as e:
            line["channel"] = {"error": repr(e)}
    if "small" in extras:
        try:
            log("small configurations")
            line["small"] = small_section()
        except Exception as e:
            line["small"] = {"error": repr(e)}
    if "precision" in extras:
        try:
            log("precision section")
            line["precision"] = precision_section(args.precision_steps)
        except Exception as e:
            line["precision"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
