"""Benchmark: one gradient of the marine 1D workload per step on one MI355X.

A step is one pass of the whole hot path for the 101x101x61 stretched-grid
marine model (3 frequencies, 1 x-dipole, 50 seabed receivers, FP32 fields
with FP64 transform accumulators): set the model, build the basis functions,
forward run with the on-the-fly receiver and volume transforms, residual
against data of the true model, adjoint run driven by the basis-function
adjoint sources with the on-the-fly gradient product, gradient on cells.

Printed: one JSON line.  value = cell updates per second over the two
simulations of the step (forward + adjoint), in Mcell-updates/s; a cell
update advances all six field components of one cell by one step.
roofline: the forward E-update kernel (fused with the volume transform),
its algorithmic bytes per launch over its average device time, from HIP
events that the sampled launches inside the timed region stamp from their
own dispatch (hipExtLaunchKernel).  cpu_baseline: the CPU
oracle stepping the same grid for a bounded window of steps.
batched_vs_plain: gradient time of the 16-source batched workload on a
window, one batched plan against one single-source plan per source.
adjoint_td: the time-domain adjoint gradient of the same step (after the
timed region) against the basis-function one.  vti: the same step on a VTI
version of the model, with the split gradient.  order4: the same step with
fourth-order differences.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    """Progress line on stderr (the JSON record is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes_e(nx, ny, nz, npml, tsize=4, kb=8, hist=True):
    """Algorithmic HBM bytes of one launch of the E update, averaged over the
    kb-step cycle of the transform block: per updated edge E read + write
    and dt/eps read (3 tsize), one H value (tsize), and, in runs with the
    volume transform or the gradient product, the sample kept in the history
    on kb-1 of kb steps ((kb-1) tsize / kb); a CPML memory variable read +
    write (2 tsize) per derivative taken inside a layer.  Returns (bytes,
    updated edges)."""
    n_ex = nx * (ny - 1) * (nz - 1)
    n_ey = (nx - 1) * ny * (nz - 1)
    n_ez = (nx - 1) * (ny - 1) * nz
    edges = n_ex + n_ey + n_ez

    def in_pml_int(n):      # interior integer nodes 1..n-1 inside a layer
        return sum(1 for i in range(1, n) if i < npml or i > n - npml)

    px, py, pz = in_pml_int(nx), in_pml_int(ny), in_pml_int(nz)
    # derivatives along y and z for E_x, x and z for E_y, x and y for E_z
    psi = (nx * py * (nz - 1) + nx * (ny - 1) * pz + px * ny * (nz - 1) + (nx - 1) * ny * pz
           + px * (ny - 1) * nz + (nx - 1) * py * nz)
    keep = (kb - 1) * tsize / kb if hist else 0.0
    return int(edges * (4 * tsize + keep) + psi * 2 * tsize), edges


def algorithmic_bytes_transform(edges, nf, tsize=4, accsize=16, kb=8, adjoint=False, blocks=None):
    """Algorithmic HBM bytes of one launch of the block transform (once per
    kb steps): per updated edge the block's kb samples (kb-1 from the
    history, the newest from the fields) and the accumulators -- forward,
    read + write of nf complex values (2 nf accsize); adjoint, a read of the
    forward transform (nf accsize) and the FP64 gradient accumulator's read
    + write (16).  The first forward block of a run only writes its
    accumulators (nf accsize): with ``blocks`` (the blocks of a run) the
    forward figure is the average over the run's launches."""
    if adjoint:
        acc = nf * accsize + 16
    elif blocks:
        acc = (2 * nf * accsize * (blocks - 1) + nf * accsize) / blocks
    else:
        acc = 2 * nf * accsize
    return int(edges * (kb * tsize + acc))


def algorithmic_bytes_e_forward(nx, ny, nz, npml, nf, tsize=4, accsize=16, kb=8):
    """The E update and the block transform of the forward run together, per
    step (the transform's bytes spread over its kb steps)."""
    be, edges = algorithmic_bytes_e(nx, ny, nz, npml, tsize, kb, True)
    return int(be + algorithmic_bytes_transform(edges, nf, tsize, accsize, kb) / kb), edges


def algorithmic_bytes_h(nx, ny, nz, npml, tsize=4):
    """Algorithmic HBM bytes of one launch of the H update: each H node read
    and written (2 tsize), each E node read once (tsize), a CPML memory
    variable read + write (2 tsize) per derivative taken inside a layer."""
    n_hx, n_hy, n_hz = (nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1)
    n_ex, n_ey, n_ez = nx * (ny + 1) * (nz + 1), (nx + 1) * ny * (nz + 1), (nx + 1) * (ny + 1) * nz

    def in_pml_half(n):     # half nodes 0..n-1 inside a layer
        return sum(1 for i in range(n) if i < npml or i >= n - npml)

    px, py, pz = in_pml_half(nx), in_pml_half(ny), in_pml_half(nz)
    # derivatives along y and z for H_x, z and x for H_y, x and y for H_z
    psi = ((nx + 1) * py * nz + (nx + 1) * ny * pz + nx * (ny + 1) * pz + px * (ny + 1) * nz
           + px * ny * (nz + 1) + nx * py * (nz + 1))
    return int((n_hx + n_hy + n_hz) * 2 * tsize + (n_ex + n_ey + n_ez) * tsize + psi * 2 * tsize)


def host_cpu_model():
    """The model line of the host CPU (lscpu's "Model name", else /proc/cpuinfo)."""
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores():
    """CPUs this process may run on, at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_slab(w, planes, k0=None):
    """A slab of ``planes`` cell layers of workload ``w`` (full x-y extent)
    holding its first source and the receivers nearest to it, with its own
    absorbing layers: a bounded sample of the workload for the CPU oracle."""
    nz = w.shape[0]
    zs = float(w.src_pos[0, 2])
    if k0 is None:
        kc = int(np.searchsorted(w.z, zs)) - 1
        k0 = max(0, min(nz - planes, kc - planes // 2))
    z = w.z[k0:k0 + planes + 1]
    inside = (w.rec_pos[:, 2] > z[w.npml + 1]) & (w.rec_pos[:, 2] < z[-w.npml - 2])
    rec = w.rec_pos[inside]
    d = np.hypot(rec[:, 0] - w.src_pos[0, 0], rec[:, 1] - w.src_pos[0, 1])
    rec = rec[np.argsort(d)[:16]]
    return w.replace(z=z, rho=np.ascontiguousarray(w.rho[k0:k0 + planes]),
                     src_pos=w.src_pos[:1], src_mom=w.src_mom[:1], rec_pos=rec,
                     name=f"{w.name}_slab{planes}")


def _oracle_gradient_window(w, steps):
    """Set up the oracle's gradient window on the one-source workload ``w``:
    returns the setup and a function that runs it -- the forward run with the
    volume transform of every frequency, then the adjoint run (basis-function
    adjoint sources, adjoint volume transform) and the gradient product, over
    ``steps`` steps each."""
    from oracle.adjoint import adjoint_sources
    from oracle.basis import basis_matrix, basis_pinv, gamma_from_rel
    from oracle.discretization import dual_volumes, make_setup
    from oracle.stepping import receiver_nodes, run_stepping, source_injection
    s = make_setup(w, nt=steps)

    def run():
        inj = source_injection(s, w.src_pos[0], w.src_mom[0])
        nodes, interp = receiver_nodes(s, w.rec_pos, w.rec_comp)
        acc, vol = run_stepping(s, inj, s.wavelet[None, :], nodes, True, steps)
        resid = np.zeros((len(w.rec_pos), len(w.rec_comp), len(s.freqs)), dtype=np.complex128)
        for r in range(len(w.rec_pos)):
            for ci in range(len(w.rec_comp)):
                resid[r, ci] = -sum(wt * acc[ni] for ni, wt in interp[r][ci]) * s.norm
        B = basis_matrix(s.a, s.dt, steps)
        b = basis_pinv(B, gamma_from_rel(B, 1e-12))
        inj_a, ts, _ = adjoint_sources(s, w.rec_pos, w.rec_comp, resid, b)
        _, v = run_stepping(s, inj_a, ts, [], True, steps)
        corr = s.Omega / s.wprime
        g = [np.real(np.einsum("k,k...->...", corr, v[c] * vol[c])) * dv
             for c, dv in enumerate(dual_volumes(s))]
        if not all(np.isfinite(x).all() for x in g):
            raise RuntimeError("oracle window produced a non-finite gradient")

    return s, run


def _cpu_worker(w, steps, barrier, out):
    """One process of the N-core leg: set up, wait for the others, run."""
    s, run = _oracle_gradient_window(w, steps)
    barrier.wait()
    t0 = time.time()
    run()
    out.put((t0, time.time(), s.nx * s.ny * s.nz))


def cpu_baseline(wname="c5_large", planes=24, steps=8):
    """The CPU oracle (NumPy FP64) on a bounded sample of the workload: a slab
    of ``planes`` cell layers (full x-y extent, one source, every frequency),
    ``steps`` forward steps with the volume transform plus ``steps`` adjoint
    steps with the gradient product -- the GPU's unit of work.  One process,
    then one process per core, each on its own copy of the slab (the slabs
    of a domain decomposition, with the halo exchange left out in the CPU's
    favour), started together after a barrier.  Runs before the GPU is
    touched (the worker processes are spawned)."""
    import multiprocessing as mp
    from workloads import by_name
    w = cpu_slab(by_name(wname), planes)
    s, run = _oracle_gradient_window(w, steps)
    cells = s.nx * s.ny * s.nz
    t0 = time.perf_counter()
    run()
    t1 = time.perf_counter() - t0
    one = 2.0 * cells * steps / t1 / 1e6
    n = host_cores()
    ctx = mp.get_context("spawn")
    barrier, out = ctx.Barrier(n), ctx.Queue()
    procs = [ctx.Process(target=_cpu_worker, args=(w, steps, barrier, out)) for _ in range(n)]
    for p in procs:
        p.start()
    res = [out.get(timeout=900) for _ in range(n)]
    for p in procs:
        p.join()
    wall = max(r[1] for r in res) - min(r[0] for r in res)
    many = 2.0 * sum(r[2] for r in res) * steps / wall / 1e6
    return {"value": many, "unit": "Mcell-updates/s", "cores": n, "kind": "oracle",
            "value_1core": one, "cpu_model": host_cpu_model(),
            "sample": f"{wname}: slab of {planes} cell layers around the first source "
                      f"({cells} cells, full x-y extent, every frequency), {steps} forward "
                      f"steps with the volume transform + {steps} adjoint steps with the "
                      f"gradient product, FP64 NumPy; one process {t1:.1f} s, then {n} "
                      f"processes on one slab each {wall:.1f} s wall"}


TILING_KEYS = ("SCHEDULE", "BLOCK_X", "BLOCK_Y", "XCD_REMAP", "VECTOR", "VECTOR_H", "TILE_ORDER",
               "ZCHUNK")


def set_tiling(plan, spec):
    from paper_2211_16665_amd import fwdem as fw
    if spec:
        for key, v in zip(TILING_KEYS, spec.split(",")):
            plan.set_option(getattr(fw, "FWD_OPT_" + key), int(v))


def measured_traffic(kernel_tag, summary, tiling=None):
    """HBM bytes per launch of a kernel from a committed counter summary
    (profiles/<summary>, lines "- traffic `<kernel>`: `<bytes>`"), or None if
    there is none, it covers no such kernel or another tiling, or the device
    source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    src = os.path.join(ROOT, "paper_2211_16665_amd", "csrc", "device.hip")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip().replace("`", "")] = v.strip().strip("`")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    key = "traffic " + kernel_tag
    if vals.get("device_source_sha256") != sha or key not in vals:
        return None
    if tiling is not None and vals.get("tiling") != tiling:
        return None
    return float(vals[key]), vals.get("tiling", "")


def batched_vs_plain(window=200):
    """Gradient time (forward with volume transform + adjoint) of the 16-source
    batched workload over a window of steps: all sources in one plan with
    graph replay, against the plain path of one single-source plan per source
    run one after the other with eager launches; FP32 fields, FP64
    accumulators, default tiling.  Then the batched plan again with the
    autotuned tiling, and its E update against its algorithmic bytes.  Also
    the largest relative gradient difference between batched and plain (the
    same arithmetic per source: 0)."""
    import torch
    from paper_2211_16665_amd import fwdem as fw
    from workloads import c4_batched, with_window
    w = with_window(c4_batched(), window)

    def gradient(plan, vol, grad):
        E, _ = plan.forward(vol=vol, want_volume=True)
        plan.adjoint(vol, -E, grad=grad, accumulate=True)

    p = fw.Plan.from_workload(w, field_dtype="f32", acc_mode="f64")
    p.set_model(w.rho)
    p.basis_build(gamma_rel=1e-12)
    vol = p.volume_buffer()
    g_b = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
    gradient(p, vol, g_b)                        # warm-up (tables, graph capture)
    g_b.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gradient(p, vol, g_b)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    del vol
    plans = []
    for s in range(w.ns):
        ws = w.replace(src_pos=w.src_pos[s:s + 1], src_mom=w.src_mom[s:s + 1])
        q = fw.Plan.from_workload(ws, field_dtype="f32", acc_mode="f64")
        q.set_option(fw.FWD_OPT_GRAPH_STEPS, 0)
        q.set_model(ws.rho)
        q.basis_build(gamma_rel=1e-12)
        plans.append((q, q.volume_buffer()))
    g_p = torch.zeros_like(g_b)
    gradient(*plans[0], torch.zeros_like(g_b))   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q, v in plans:
        gradient(q, v, g_p)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    diff = float((g_b - g_p).abs().max() / g_p.abs().max())
    nz, ny, nx = p.shape
    # the batched plan with the autotuned tiling, then its E update against
    # its algorithmic bytes: per source as in the single-source model, dt/eps
    # read once per launch for all sources
    del plans
    vol = p.volume_buffer()
    p.autotune(fw.FWD_MODE_FORWARD, vol=vol, steps=16)
    tuned = {k.lower(): int(p.get_option(getattr(fw, "FWD_OPT_" + k))) for k in TILING_KEYS}
    gradient(p, vol, g_b)                        # warm-up with the tuned tiling
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gradient(p, vol, g_b)
    torch.cuda.synchronize()
    t_tuned = time.perf_counter() - t0
    p.set_option(fw.FWD_OPT_SAMPLE_EVERY, 64)
    p.forward(vol=vol, want_volume=True)
    kb = int(p.get_option(fw.FWD_OPT_DFT_BLOCK))
    kern = kernel_records([p.kernel_stats()], w.ns, nx, ny, nz, w.npml, len(w.freqs), 4, 16,
                          kb, "F64", max(1, window // kb))
    del vol
    return {"workload": f"c4_batched window: {nx}x{ny}x{nz}, {w.ns} sources, {len(w.freqs)} freqs, "
                        f"{window} forward + {window} adjoint steps",
            "batched_s": t_batched, "plain_s": t_plain, "speedup": t_plain / t_batched,
            "batched_tuned_s": t_tuned, "speedup_tuned": t_plain / t_tuned, "tuning": tuned,
            "kernels_ms": kern,
            "batched_mcell_per_s": 2 * w.ns * nx * ny * nz * window / t_batched / 1e6,
            "max_rel_grad_diff": diff}


def reciprocity_study(window=200):
    """The reciprocity swap on a towline survey like the paper's marine
    example (Section 4: many sources, few receivers): the marine grid with 81
    x-dipoles every 75 m along the tow line and 2 seabed receivers (E_x,
    E_y), a gradient window of ``window`` forward + ``window`` adjoint steps
    (FP32 fields, FP64 accumulators), the 81 sources batched in one plan
    against the 4 swapped runs (one unit dipole per receiver component).
    Also the largest relative difference of the data (exact reciprocity:
    rounding only).  The window is too short for the adjoint sources' basis
    to fit well, so only times are compared for the adjoint; the gradient
    identity is checked in the tests."""
    import torch
    from paper_2211_16665_amd import fwdem as fw
    from paper_2211_16665_amd.reciprocity import fields_to_data, swap_workload
    from workloads import c2_marine1d, with_window
    xs = np.arange(-3000.0, 3000.0 + 1.0, 75.0)
    src = np.stack([xs, np.zeros_like(xs), np.full_like(xs, 250.0)], axis=1)
    w = with_window(c2_marine1d(), window).replace(
        src_pos=src, src_mom=np.tile([1.0, 0.0, 0.0], (len(xs), 1)),
        rec_pos=np.array([[-500.0, 0.0, 300.0], [500.0, 0.0, 300.0]]), rec_comp=(0, 1))
    ws = swap_workload(w)

    def gradient_time(wk):
        p = fw.Plan.from_workload(wk, field_dtype="f32", acc_mode="f64")
        p.set_model(wk.rho)
        p.basis_build(gamma_rel=1e-12)
        vol = p.volume_buffer()
        g = torch.zeros(p.shape, dtype=torch.float64, device="cuda")

        def run():
            E, _ = p.forward(vol=vol, want_volume=True)
            p.adjoint(vol, -E, grad=g, accumulate=True)
            return E

        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E = run()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        E = E.cpu().numpy()
        del p, vol, g
        torch.cuda.empty_cache()
        return t, E

    t_o, E_o = gradient_time(w)
    t_s, E_s = gradient_time(ws)
    d_s = fields_to_data(E_s, w.src_mom, len(w.rec_comp))
    return {"workload": f"c2_marine1d towline: {len(xs)} x-dipoles, 2 seabed receivers (E_x, E_y), "
                        f"{window} forward + {window} adjoint steps",
            "original_s": t_o, "swapped_s": t_s, "speedup": t_o / t_s,
            "original_sources": len(w.src_pos), "swapped_sources": len(ws.src_pos),
            "max_rel_data_diff": float(np.abs(d_s - E_o).max() / np.abs(E_o).max())}


def vti_study(plan, w_true, rho0, iso_s):
    """The same gradient step on a VTI version of the marine model (vertical
    resistivity twice the horizontal one below the sea floor), with the split
    gradient: time against the isotropic step (same kernels; only the edge
    conductivities and the gradient scatter differ)."""
    import torch
    from paper_2211_16665_amd import fwdem as fw
    from workloads import with_vti
    wv = with_vti(w_true, ratio=2.0)
    plan.set_model(wv.rho, wv.rho_v)
    d_obs = plan.forward()
    rv0 = rho0.copy()
    rv0[rho0 >= 0.9] *= 2.0
    plan.set_option(fw.FWD_OPT_VTI_GRADIENT, 1)
    vol = plan.volume_buffer()
    grad = torch.zeros(plan.grad_shape, dtype=torch.float64, device="cuda")

    def step():
        plan.set_model(rho0, rv0)
        plan.basis_build(gamma_rel=1e-12)
        E, _ = plan.forward(vol=vol, want_volume=True)
        plan.adjoint(vol, d_obs - E, grad=grad)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    plan.set_option(fw.FWD_OPT_VTI_GRADIENT, 0)
    g = grad.abs().amax(dim=(1, 2, 3)).tolist()
    return {"model": "c2_marine1d with rho_v = 2 rho_h below the sea floor", "gradient_s": t,
            "isotropic_gradient_s": iso_s, "nt": plan.info.nt,
            "max_abs_grad_h": g[0], "max_abs_grad_v": g[1]}


def magnetic_study(w_true, rho0, tuned, electric_s):
    """The same gradient step with magnetic data: receivers recording E_x,
    E_y, H_x, H_y (a plan of its own, with the tiling of the main plan).
    The H transform and the magnetic adjoint source run as one small kernel
    per step each, beside the step's own kernels; the time against the
    electric-only step measures their cost."""
    import torch
    from paper_2211_16665_amd import fwdem as fw
    wm = w_true.replace(rec_comp=(0, 1, 3, 4))
    plan = fw.Plan.from_workload(wm, field_dtype="f32", acc_mode="f64")
    for k in TILING_KEYS:
        plan.set_option(getattr(fw, "FWD_OPT_" + k), tuned[k.lower()])
    plan.set_model(wm.rho)
    d_obs = plan.forward()
    vol = plan.volume_buffer()
    grad = torch.zeros(plan.shape, dtype=torch.float64, device="cuda")

    plan.set_option(fw.FWD_OPT_SAMPLE_EVERY, 2048)
    ks = []

    def step():
        plan.set_model(rho0)
        plan.basis_build(gamma_rel=1e-12)
        E, _ = plan.forward(vol=vol, want_volume=True)
        ks.append(plan.kernel_stats())
        plan.adjoint(vol, d_obs - E, grad=grad)
        ks.append(plan.kernel_stats())

    step()
    ks.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out = {"receivers": "E_x, E_y, H_x, H_y", "gradient_s": t, "electric_gradient_s": electric_s,
           "overhead": t / electric_s - 1.0, "rec_nodes": plan.info.n_rec_nodes,
           "kernels_ms": {"update_h": {"fwd_ms": ks[0][0][0], "adj_ms": ks[1][0][0]},
                          "update_e": {"fwd_ms": ks[0][0][1], "adj_ms": ks[1][0][1]},
                          "transform": {"fwd_ms": ks[0][0][2], "adj_ms": ks[1][0][2]}}}
    del plan, vol, grad
    torch.cuda.empty_cache()
    return out


def order4_study(w_true, rho0, order2_s, tsize, accsize):
    """The same gradient step with fourth-order differences (a plan of its
    own: the order changes dt, nt and the tables): time against the
    second-order step, and the order-4 kernels against the same algorithmic
    bytes (each field value is still read and written once per step)."""
    import torch
    from paper_2211_16665_amd import fwdem as fw
    w4 = w_true.replace(fd_order=4)
    plan = fw.Plan.from_workload(w4, field_dtype="f32", acc_mode="f64")
    plan.set_model(w4.rho)
    d_obs = plan.forward()
    vol = plan.volume_buffer()
    plan.autotune(fw.FWD_MODE_FORWARD, vol=vol, steps=16)
    plan.set_option(fw.FWD_OPT_SAMPLE_EVERY, 2048)
    grad = torch.zeros(plan.shape, dtype=torch.float64, device="cuda")
    ks = []

    def step():
        plan.set_model(rho0)
        plan.basis_build(gamma_rel=1e-12)
        E, _ = plan.forward(vol=vol, want_volume=True)
        ks.append(plan.kernel_stats())
        plan.adjoint(vol, d_obs - E, grad=grad)

    step()
    ks.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    nz, ny, nx = plan.shape
    kb = int(plan.get_option(fw.FWD_OPT_DFT_BLOCK))
    kern = kernel_records(ks[:1], 1, nx, ny, nz, w_true.npml, len(w_true.freqs), tsize, accsize,
                          kb, "F64", max(1, plan.info.nt // kb))
    nt = plan.info.nt
    out = {"gradient_s": t, "order2_gradient_s": order2_s, "nt": nt, "dt": plan.info.dt,
           "mcell_per_s": 2.0 * nx * ny * nz * nt / t / 1e6,
           "tiling": {k.lower(): int(plan.get_option(getattr(fw, "FWD_OPT_" + k)))
                      for k in ("BLOCK_X", "BLOCK_Y", "XCD_REMAP", "TILE_ORDER")},
           "kernels_ms": kern}
    del plan, vol, grad
    torch.cuda.empty_cache()
    return out


def decimation_study(plan, rho0, d_obs, vol, exact_s, factors=(8, 64)):
    """The marine gradient with the forward volume transform decimated by D
    (every D-th sample, weight D; receivers and the adjoint product keep
    every sample): seconds per gradient and the gradient's relative L2
    difference to the exact one."""
    import torch
    from paper_2211_16665_amd import fwdem as fw

    def gradient():
        plan.set_model(rho0)
        plan.basis_build(gamma_rel=1e-12)
        E, _ = plan.forward(vol=vol, want_volume=True)
        return plan.adjoint(vol, d_obs - E)

    g1 = gradient()
    out = {"exact_s": exact_s}
    for D in factors:
        plan.set_option(fw.FWD_OPT_DFT_DECIMATE, D)
        gradient()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = gradient()
        torch.cuda.synchronize()
        out[f"D{D}"] = {"gradient_s": time.perf_counter() - t0,
                        "gradient_rel_l2_vs_exact": float((g - g1).norm() / g1.norm())}
    plan.set_option(fw.FWD_OPT_DFT_DECIMATE, 1)
    return out


def schedules_study(tuned, window=2000):
    """The three schedules on a window of the marine workload (its first
    ``window`` steps, FP32 fields, receiver and volume transforms): time per
    step of the tuned two-kernel schedule, the fused schedule (one launch per
    step) and the persistent schedule (one cooperative launch; at the
    occupancy-sized grid and at one block per compute unit), each checked
    bit for bit against the two-kernel receivers."""
    import numpy as np
    import torch
    from paper_2211_16665_amd import fwdem as fw
    from workloads import c2_marine1d, with_window
    w = with_window(c2_marine1d(), window)
    kb = tuned["dft_block"] if tuned["dft_block"] in (8, 16) else 8

    def per_step(opts):
        p = fw.Plan.from_workload(w, field_dtype="f32", acc_mode="f64")
        for k, v in opts.items():
            p.set_option(getattr(fw, "FWD_OPT_" + k), v)
        p.set_model(w.rho)
        vol = p.volume_buffer()
        p.forward(vol=vol, want_volume=True)            # warm-up (graphs, lists)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E, _ = p.forward(vol=vol, want_volume=True)
        torch.cuda.synchronize()
        us = (time.perf_counter() - t0) / window * 1e6
        return us, E.cpu().numpy()

    base = {k.upper(): tuned[k.lower()] for k in TILING_KEYS}
    base["DFT_BLOCK"] = kb
    us0, E0 = per_step(base)
    out = {"window": window, "dft_block": kb, "two_kernel_tuned_us_per_step": us0}
    runs = (("fused_64x4", dict(SCHEDULE=1, BLOCK_X=64, BLOCK_Y=4, ZCHUNK=4)),
            ("fused_32x8", dict(SCHEDULE=1, BLOCK_X=32, BLOCK_Y=8, ZCHUNK=4)),
            ("persistent_64x4", dict(SCHEDULE=2, BLOCK_X=64, BLOCK_Y=4)),
            ("persistent_64x4_1_block_per_cu", dict(SCHEDULE=2, BLOCK_X=64, BLOCK_Y=4,
                                                    PERSIST_BLOCKS=1)))
    for name, opts in runs:
        opts = dict(opts, VECTOR=1, VECTOR_H=1, XCD_REMAP=0, DFT_BLOCK=kb)
        us, E = per_step(opts)
        out[name] = {"us_per_step": us, "receivers_bitwise_equal": bool(np.array_equal(E, E0))}
        log(f"schedules: {name} {out[name]}")
    return out


def adjoint_td_study(plan, resid, grad_basis, basis_s, npml, segment=500):
    """The time-domain adjoint (Appendix) on the bench workload: gradient time
    (forward with checkpoints, replay, reverse sweep) against the
    basis-function gradient of the timed step, and their agreement outside
    the CPML layers (inside them only the time-domain gradient is the
    derivative of the stepped system)."""
    import torch
    scratch = torch.empty(plan.adjoint_td_size(segment), dtype=torch.uint8, device="cuda")
    plan.adjoint_td(resid, segment=segment, scratch=scratch)          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = plan.adjoint_td(resid, segment=segment, scratch=scratch)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    inner = (slice(npml, -npml),) * 3
    gb = grad_basis[inner]
    diff = float((g[inner] - gb).norm() / gb.norm())
    nz, ny, nx = plan.shape
    return {"segment": segment, "gradient_s": t, "basis_gradient_s": basis_s,
            "scratch_gb": scratch.numel() / 1e9,
            "mcell_per_s_three_sweeps": 3.0 * plan.ns * nx * ny * nz * plan.info.nt / t / 1e6,
            "rel_l2_vs_basis_outside_cpml": diff}


def background_model(w):
    """The start model of the gradient step: the true model with its
    100 ohm-m reservoir cells replaced by 1 ohm-m sediment."""
    rho0 = w.rho.copy()
    rho0[rho0 == 100.0] = 1.0
    return rho0


def kernel_records(stats, ns, nx, ny, nz, npml, nf, tsize, accsize, kb, acc_tag, blocks):
    """Per kernel of a forward step (H update, E update, block transform):
    the average launch time over the sampled steps of the forward runs in
    ``stats`` (kernel_stats() results), its algorithmic bytes per launch for
    ``ns`` sources (dt/eps read once for all of them; the transform's
    averaged over the ``blocks`` blocks of a run) and the time per step (the
    block transform runs once in kb steps)."""
    ok = [s_ for s_ in stats if s_[1] > 0]
    ms = [float(np.mean([s_[0][k] for s_ in ok])) if ok else float("nan") for k in range(3)]
    samples = sum(s_[1] for s_ in stats)
    per_e, edges = algorithmic_bytes_e(nx, ny, nz, npml, tsize, kb, True)
    t = "float" if tsize == 4 else "double"
    out = {
        "update_h": {"kernel": f"k_update_h<{t}>",
                     "bytes_per_launch": ns * algorithmic_bytes_h(nx, ny, nz, npml, tsize),
                     "avg_launch_ms": ms[0], "ms_per_step": ms[0]},
        "update_e": {"kernel": f"k_update_e<{t},hist>",
                     "bytes_per_launch": ns * per_e - (ns - 1) * edges * tsize,
                     "avg_launch_ms": ms[1], "ms_per_step": ms[1]},
        "transform": {"kernel": f"k_transform<{t},{acc_tag},fwd,{kb}>",
                      "bytes_per_launch": ns * algorithmic_bytes_transform(edges, nf, tsize,
                                                                           accsize, kb,
                                                                           blocks=blocks),
                      "avg_launch_ms": ms[2], "ms_per_step": ms[2] / kb},
    }
    for v in out.values():
        v["samples"] = samples
        v["algorithmic_gbs"] = v["bytes_per_launch"] / (v["avg_launch_ms"] * 1e-3) / 1e9
        v["frac_of_hbm_peak"] = v["algorithmic_gbs"] / HBM_PEAK_GBS
    return out


def source_groups(ns, per_source_bytes, free_bytes, frac=0.8):
    """Split ``ns`` sources into groups of near-equal size whose workspace and
    volume transform fit in ``frac`` of the free device memory."""
    g = max(1, min(ns, int(frac * free_bytes // per_source_bytes)))
    ng = -(-ns // g)
    base, extra = divmod(ns, ng)
    sizes = [base + (1 if i < extra else 0) for i in range(ng)]
    out, s0 = [], 0
    for n in sizes:
        out.append((s0, s0 + n))
        s0 += n
    return out


def large_window(args):
    """The headline: one gradient window of the 400x400x200 workload (32M
    cells, 8 frequencies, 32 x-dipoles, 400 seabed receivers).  The sources
    run in groups sized to the device memory (one plan per group, all
    sources of a group advanced together in every launch, one shared
    workspace and volume buffer); a step is, for every group, the forward
    run with the receiver and volume transforms and the adjoint run of the
    window's misfit 1/2 |E|^2 with the gradient product, accumulated into
    one gradient.  The model and the basis functions are set up once,
    untimed (over a full-length run they are a one-time cost)."""
    import torch
    from paper_2211_16665_amd import fwdem as fw
    from workloads import c5_large, with_window
    t_setup = time.perf_counter()
    w = with_window(c5_large(), args.window)
    acc = args.acc or w.acc_mode
    rho0 = background_model(w)
    # workspaces sized for the longest transform block (32 samples), so that
    # the autotuner may choose any block
    one = fw.Plan.from_workload(w.replace(src_pos=w.src_pos[:1], src_mom=w.src_mom[:1]),
                                field_dtype=args.field_dtype, acc_mode=acc)
    one.set_option(fw.FWD_OPT_DFT_BLOCK, 32)
    one.set_model(w.rho)
    per_src = one.workspace_size(fw.FWD_MODE_ADJOINT) + one.volume_size()
    del one
    free, total = torch.cuda.mem_get_info()
    groups = source_groups(w.ns, per_src, free) if not args.group else \
        [(a, min(a + args.group, w.ns)) for a in range(0, w.ns, args.group)]
    plans = []
    for a, b in groups:
        wg = w.replace(src_pos=w.src_pos[a:b], src_mom=w.src_mom[a:b])
        p = fw.Plan.from_workload(wg, field_dtype=args.field_dtype, acc_mode=acc)
        p.set_option(fw.FWD_OPT_DFT_BLOCK, 32)
        p.set_model(w.rho)
        plans.append(p)
    gmax = max(b - a for a, b in groups)
    big = max(range(len(plans)), key=lambda i: groups[i][1] - groups[i][0])
    ws = torch.empty(plans[big].workspace_size(fw.FWD_MODE_ADJOINT), dtype=torch.uint8,
                     device="cuda")
    vol = torch.empty(plans[big].volume_size(), dtype=torch.uint8, device="cuda")
    for p in plans:
        p.use_workspace(ws)
    log(f"large workload: {len(groups)} groups {[b - a for a, b in groups]}, "
        f"{per_src / 1e9:.1f} GB per source, {free / 1e9:.0f} GB free")
    if args.tiling:
        set_tiling(plans[big], args.tiling)
        if args.dft_block:
            plans[big].set_option(fw.FWD_OPT_DFT_BLOCK, args.dft_block)
        tune_ms = float("nan")
    else:
        tune_ms = plans[big].autotune(fw.FWD_MODE_FORWARD, vol=vol, steps=args.tune_steps)
    tuned = {k.lower(): int(plans[big].get_option(getattr(fw, "FWD_OPT_" + k)))
             for k in TILING_KEYS + ("DFT_BLOCK",)}
    for p in plans:
        for k in TILING_KEYS + ("DFT_BLOCK",):
            p.set_option(getattr(fw, "FWD_OPT_" + k), tuned[k.lower()])
        p.set_model(rho0)
        p.basis_build(gamma_rel=1e-12)
        p.set_option(fw.FWD_OPT_SAMPLE_EVERY, args.sample_every)
    tuned["ms_per_forward_step"] = tune_ms
    grad = torch.zeros(plans[0].shape, dtype=torch.float64, device="cuda")
    stats = []

    def step():
        for gi, p in enumerate(plans):
            E, _ = p.forward(vol=vol, want_volume=True)
            if p is plans[big]:
                stats.append(p.kernel_stats())
            # the misfit 1/2 |E|^2 of the window's own receiver fields: over
            # the first steps of a run the data of the true model differ
            # from the prediction by nothing the receivers can see yet (the
            # reservoir is thousands of steps of travel away), which would
            # make the adjoint sources zero
            p.adjoint(vol, -E, grad=grad, accumulate=gi > 0)

    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    log(f"setup {t_setup:.1f} s (tuning {tuned})")
    for _ in range(args.warmup):
        step()
    stats.clear()
    torch.cuda.synchronize()
    log("warm-up done")
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        if i % 5 == 4 or i == args.steps - 1:
            log(f"step {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if not torch.isfinite(grad).all():
        raise RuntimeError("non-finite gradient")
    headline_stats = list(stats)
    decimated = None
    if args.decimate > 1:
        # the same window with the forward volume transform decimated (an
        # approximation, not the headline): time and gradient against the
        # exact one
        g_exact = grad.clone()
        for p in plans:
            p.set_option(fw.FWD_OPT_DFT_DECIMATE, args.decimate)
        step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        dt_dec = time.perf_counter() - t1
        if not torch.isfinite(grad).all():
            raise RuntimeError("non-finite gradient with a decimated volume transform")
        err = float((grad - g_exact).norm() / g_exact.norm())
        decimated = {"decimate": args.decimate, "ms_per_step": dt_dec * 1e3,
                     "speedup": elapsed / args.steps / dt_dec,
                     "gradient_rel_l2_vs_exact": err,
                     "gradient_norm": float(g_exact.norm())}
        for p in plans:
            p.set_option(fw.FWD_OPT_DFT_DECIMATE, 1)
        log(f"decimated by {args.decimate}: {dt_dec * 1e3:.0f} ms per step, gradient {err:.1e}")
    nz, ny, nx = plans[0].shape
    ncells = nx * ny * nz
    updates = 2.0 * w.ns * ncells * args.window * args.steps
    tsize = 4 if args.field_dtype == "f32" else 8
    accsize = 8 if acc == "f32" else 16
    kb = tuned["dft_block"]
    nf = len(w.freqs)
    kern = kernel_records(headline_stats, gmax, nx, ny, nz, w.npml, nf, tsize, accsize, kb,
                          "KAHAN" if acc == "kahan" else acc.upper(), max(1, args.window // kb))
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
    mt = measured_traffic(kern[dom]["kernel"], "pmc_large_step_kernels.md",
                          ",".join(str(tuned[k.lower()]) for k in TILING_KEYS))
    desc = (f"c5_large gradient window: 400x400x200 stretched grid (100 m core, ratio 1.05), "
            f"random log-normal sediment (corr. 500 m) with a 100 ohm-m 2x2 km reservoir, "
            f"8 freqs 0.1-2 Hz, {w.ns} x-dipoles in {len(groups)} groups of <= {gmax} "
            f"(one plan per group, sources of a group batched in every launch), "
            f"400 seabed receivers; {args.window} forward + {args.window} adjoint steps with "
            f"receiver and volume transforms and the gradient product (misfit 1/2 |E|^2 of "
            f"the window's receivers), summed over groups")
    out = {
        "metric": "Mcell-updates/s",
        "value": updates / elapsed / 1e6,
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.field_dtype,
        "data": "synthetic",
        "config": {"workload": desc, "cells": ncells, "window_steps": args.window,
                   "dt": plans[0].info.dt, "sources": w.ns,
                   "groups": [b - a for a, b in groups], "field_dtype": args.field_dtype,
                   "accumulators": acc, "tuning": tuned,
                   "setup_s": t_setup,
                   "device_bytes_per_source": per_src},
        "roofline": {"bound": "hbm", "achieved": kern[dom]["algorithmic_gbs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": kern[dom]["algorithmic_gbs"] / HBM_PEAK_GBS,
                     "traffic": mt[0] if mt else None, "kernel": kern[dom]["kernel"],
                     "tiling": ",".join(str(tuned[k.lower()]) for k in TILING_KEYS),
                     "sources_per_launch": gmax,
                     "bytes_per_launch": kern[dom]["bytes_per_launch"],
                     "avg_launch_ms": kern[dom]["avg_launch_ms"],
                     "samples": kern[dom]["samples"]},
        "kernels_ms": kern,
    }
    if decimated is not None:
        out["decimated_volume_transform"] = decimated
    del plans, ws, vol, grad
    torch.cuda.empty_cache()
    return out


def marine_gradient(args):
    """The full gradient of the 101x101x61 marine workload (every one of its
    steps), the configuration the oracle checks end to end.  Its working set
    (~110 MB) lives in the 256 MB Infinity Cache, so its roofline is that of
    the last-level cache, not HBM.  Returns the record and what the studies
    that reuse its plan need."""
    import torch
    from paper_2211_16665_amd import fwdem as fw
    from workloads import c2_marine1d
    w_true = c2_marine1d().replace(fd_order=args.fd_order)
    rho0 = background_model(w_true)
    plan = fw.Plan.from_workload(w_true, field_dtype=args.field_dtype, acc_mode=args.acc or "f64")
    plan.set_model(w_true.rho)
    d_obs = plan.forward()
    vol = plan.volume_buffer()
    tune_ms = plan.autotune(fw.FWD_MODE_FORWARD, vol=vol, steps=32)
    tuned = {k.lower(): int(plan.get_option(getattr(fw, "FWD_OPT_" + k)))
             for k in TILING_KEYS + ("DFT_BLOCK",)}
    tuned["ms_per_forward_step"] = tune_ms
    grad = torch.zeros(plan.shape, dtype=torch.float64, device="cuda")
    stats = []
    resid_last = []

    def step():
        plan.set_model(rho0)
        plan.basis_build(gamma_rel=1e-12)
        E, _ = plan.forward(vol=vol, want_volume=True)
        stats.append(plan.kernel_stats())
        resid = d_obs - E
        resid_last[:] = [resid]
        plan.adjoint(vol, resid, grad=grad)

    # timed with no kernel sampling (each sampled step runs eagerly with
    # events, ~0.6 ms extra on this small grid); one sampled step afterwards
    # gives the kernel times
    plan.set_option(fw.FWD_OPT_SAMPLE_EVERY, 0)
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.marine_steps):
        step()
    torch.cuda.synchronize()
    elapsed = (time.perf_counter() - t0) / args.marine_steps
    plan.set_option(fw.FWD_OPT_SAMPLE_EVERY, args.sample_every)
    stats.clear()
    step()
    plan.set_option(fw.FWD_OPT_SAMPLE_EVERY, 0)
    nz, ny, nx = plan.shape
    nt = plan.info.nt
    tsize = 4 if args.field_dtype == "f32" else 8
    accsize = 8 if args.acc == "f32" else 16
    kb = tuned["dft_block"]
    kern = kernel_records(stats, 1, nx, ny, nz, w_true.npml, len(w_true.freqs), tsize, accsize,
                          kb, "F64", max(1, nt // kb))
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
    mt = measured_traffic(kern[dom]["kernel"], "pmc_marine1d_e_update.md")
    out = {"workload": "c2_marine1d gradient: 101x101x61 stretched grid, 3 freqs, 1 x-dipole, "
                       "50 seabed receivers; full forward + adjoint + gradient "
                       "(setting the model and the basis functions included)",
           "gradient_s": elapsed, "nt": nt, "cells": nx * ny * nz,
           "mcell_per_s": 2.0 * nx * ny * nz * nt / elapsed / 1e6, "tuning": tuned,
           "basis_fit": plan.info.basis_fit,
           "roofline": {"bound": "llc", "achieved": kern[dom]["algorithmic_gbs"],
                        "unit": "GB/s", "kernel": kern[dom]["kernel"],
                        "bytes_per_launch": kern[dom]["bytes_per_launch"],
                        "avg_launch_ms": kern[dom]["avg_launch_ms"],
                        "frac_of_hbm_peak": kern[dom]["frac_of_hbm_peak"],
                        "traffic": mt[0] if mt else None,
                        "note": "working set ~110 MB, resident in the 256 MB Infinity Cache"},
           "kernels_ms": kern}
    return out, plan, w_true, rho0, resid_last[0], grad, vol, tuned


def profile_mode(args):
    """A short run for hardware-counter collection: one elementwise kernel of
    a known size (1 GiB read + 1 GiB written, the calibration of the byte
    counters; larger than the 256 MB Infinity Cache), two more calibration
    points (a 256 MiB elementwise kernel, a 1 GiB reduction), then a forward
    and an adjoint run of ``profile_steps`` steps on the full grid of the
    workload (for the large workload: one group of ``--group`` sources), with
    eager launches."""
    import torch
    from paper_2211_16665_amd import fwdem as fw
    from workloads import c2_marine1d, c4_batched, c5_large
    n = 1024 * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.mul(a, 2.0, out=b)          # one elementwise kernel: 1 GiB read, 1 GiB written
    torch.cuda.synchronize()
    # two more calibration points: a 256 MiB elementwise kernel, and a
    # reduction that reads 1 GiB and writes almost nothing
    q = n // 4
    torch.mul(a[:q], 3.0, out=b[:q])
    torch.cuda.synchronize()
    r = torch.sum(a)
    torch.cuda.synchronize()
    del a, b, r
    if args.profile_workload == "large":
        w = c5_large()
        g = args.group or 8
        w = w.replace(src_pos=w.src_pos[:g], src_mom=w.src_mom[:g])
    elif args.profile_workload == "batched":
        w = c4_batched()
    else:
        w = c2_marine1d().replace(fd_order=args.fd_order)
    w = w.replace(nt=args.profile_steps)
    plan = fw.Plan.from_workload(w, field_dtype=args.field_dtype, acc_mode=args.acc or w.acc_mode)
    plan.set_option(fw.FWD_OPT_GRAPH_STEPS, 0)
    set_tiling(plan, args.tiling)
    if args.dft_block:
        plan.set_option(fw.FWD_OPT_DFT_BLOCK, args.dft_block)
    plan.set_model(w.rho)
    plan.basis_build(gamma_rel=1e-12)
    E, vol = plan.forward(want_volume=True)
    plan.adjoint(vol, -E)
    if args.profile_td > 0:
        # the time-domain adjoint of the same run, checkpoints every
        # profile_td steps
        plan.adjoint_td(-E, segment=args.profile_td)
    torch.cuda.synchronize()
    print(json.dumps({"profile_steps": args.profile_steps, "copy_bytes": 4 * n,
                      "workload": w.name, "sources": w.ns}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--window", type=int, default=64,
                    help="forward (and adjoint) steps of the large workload's gradient window")
    ap.add_argument("--group", type=int, default=0,
                    help="sources per plan of the large workload (0: sized to the memory)")
    ap.add_argument("--tune-steps", type=int, default=16)
    ap.add_argument("--marine-steps", type=int, default=3,
                    help="timed full gradients of the marine workload (extra record)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--field-dtype", default="f32")
    ap.add_argument("--acc", default="",
                    help="volume accumulators f64 / kahan / f32 (default: the workload's)")
    ap.add_argument("--sample-every", type=int, default=64)
    ap.add_argument("--no-marine", action="store_true",
                    help="skip the marine workload's full gradient and the studies built on it")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-vs-plain gradient-time comparison")
    ap.add_argument("--no-schedules", action="store_true",
                    help="skip the fused and persistent schedules' timing on the marine step")
    ap.add_argument("--no-td", action="store_true",
                    help="skip the time-domain adjoint study")
    ap.add_argument("--no-vti", action="store_true",
                    help="skip the VTI gradient timing")
    ap.add_argument("--fd-order", type=int, default=2, choices=(2, 4),
                    help="order of the staggered differences of the marine step")
    ap.add_argument("--no-reciprocity", action="store_true",
                    help="skip the towline study of the source-receiver swap")
    ap.add_argument("--no-magnetic", action="store_true",
                    help="skip the gradient step with magnetic receivers")
    ap.add_argument("--no-order4", action="store_true",
                    help="skip the fourth-order gradient timing")
    ap.add_argument("--extras", default="all",
                    help="'none' skips every extra record (marine, studies, CPU baseline)")
    ap.add_argument("--decimate", type=int, default=16,
                    help="also time the headline window with the forward volume transform "
                         "decimated by this factor (1: skip); never the headline value")
    ap.add_argument("--dft-block", type=int, default=0,
                    help="with --tiling: the transform block (0: the plan's default)")
    ap.add_argument("--tiling", default="",
                    help="fixed tiling instead of autotuning: " + ",".join(TILING_KEYS).lower())
    ap.add_argument("--profile-workload", default="large", choices=("large", "marine", "batched"),
                    help="workload of the counter-collection mode")
    ap.add_argument("--profile-td", type=int, default=0,
                    help="counter-collection mode: also the time-domain adjoint, with "
                         "checkpoints every this many steps")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="counter-collection mode: a 1 GiB device copy (calibration of the "
                         "byte counters) then this many forward and adjoint steps of the "
                         "workload; prints a short JSON line, no metric")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the path has no multi-GPU mode "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)
    if args.extras == "none":
        args.no_cpu = args.no_marine = args.no_batched = args.no_reciprocity = True

    # the CPU leg first: its worker processes are started before anything
    # touches the GPU
    cpu = None if args.no_cpu or args.profile_steps > 0 else cpu_baseline()
    if cpu is not None:
        log(f"CPU baseline: {cpu['value']:.1f} Mcell-updates/s on {cpu['cores']} cores")

    import torch
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.profile_steps > 0:
        profile_mode(args)
        return
    out = large_window(args)
    log(f"headline: {out['value']:.0f} Mcell-updates/s, {out['ms_per_step']:.0f} ms per step")
    if not args.no_marine:
        marine, plan, w_true, rho0, resid, grad, vol, tuned = marine_gradient(args)
        out["marine1d"] = marine
        base_s = marine["gradient_s"]
        tsize = 4 if args.field_dtype == "f32" else 8
        if not args.no_schedules:
            out["schedules"] = schedules_study(tuned)
        if args.decimate > 1:
            out["marine_decimation"] = decimation_study(plan, rho0, resid + plan.forward(), vol,
                                                        base_s)
        if not args.no_td:
            out["adjoint_td"] = adjoint_td_study(plan, resid, grad, base_s, w_true.npml)
        if not args.no_vti:             # changes the plan's model: after the studies above
            out["vti"] = vti_study(plan, w_true, rho0, base_s)
        del plan, vol, grad
        torch.cuda.empty_cache()
        if not args.no_order4 and args.fd_order == 2:
            out["order4"] = order4_study(w_true, rho0, base_s, tsize, 16)
        if not args.no_magnetic and args.fd_order == 2 and args.field_dtype == "f32":
            out["magnetic"] = magnetic_study(w_true, rho0, tuned, base_s)
    if not args.no_batched:
        torch.cuda.empty_cache()
        out["batched_vs_plain"] = batched_vs_plain()
    if not args.no_reciprocity:
        out["reciprocity"] = reciprocity_study()
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
