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


def algorithmic_bytes_e_forward(nx, ny, nz, npml, nf, tsize=4, accsize=16, kb=8):
    """Algorithmic HBM bytes of one launch of the forward E update fused with
    the volume transform, averaged over the kb-step cycle of the transform
    block: per updated edge E read + write and dt/eps read (3 tsize), one H
    value (tsize), the accumulator read-modify-write of nf complex values
    once per cycle (2 nf accsize / kb), the history of the cycle (kb-2
    samples written once and read once: 2 (kb-2) tsize / kb); a CPML memory
    variable read + write (2 tsize) per derivative taken inside a layer."""
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
    hist = 2 * max(kb - 2, 0) * tsize / kb
    per_edge = 4 * tsize + 2 * nf * accsize / kb + hist
    return int(edges * per_edge + psi * 2 * tsize), edges


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


def cpu_baseline(w, steps=400):
    """Oracle (NumPy FP64, single process) stepping the full grid of the
    workload with the volume transform for a bounded window of steps."""
    import oracle
    from oracle.discretization import make_setup
    from oracle.stepping import receiver_nodes, run_stepping, source_injection
    s = make_setup(w, nt=steps)
    inj = source_injection(s, w.src_pos[0], w.src_mom[0])
    nodes, _ = receiver_nodes(s, w.rec_pos, w.rec_comp)
    t0 = time.perf_counter()
    run_stepping(s, inj, s.wavelet[None, :], nodes, True, steps)
    dt = time.perf_counter() - t0
    ncells = s.nx * s.ny * s.nz
    return {"value": ncells * steps / dt / 1e6, "unit": "Mcell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{w.name}: full {s.nx}x{s.ny}x{s.nz} grid, {steps} forward steps with "
                      f"the volume transform of {len(s.freqs)} frequencies, FP64 NumPy, "
                      f"one process ({dt:.1f} s); host {os.cpu_count()} logical CPUs"}


TILING_KEYS = ("SCHEDULE", "BLOCK_X", "BLOCK_Y", "XCD_REMAP", "VECTOR", "VECTOR_H", "TILE_ORDER",
               "ZCHUNK")


def set_tiling(plan, spec):
    from paper_2211_16665_amd import fwdem as fw
    if spec:
        for key, v in zip(TILING_KEYS, spec.split(",")):
            plan.set_option(getattr(fw, "FWD_OPT_" + key), int(v))


def measured_traffic(kernel_tag):
    """HBM bytes per launch of a kernel from the committed counter summary
    (profiles/), or None if the device source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_marine1d_e_update.md")
    src = os.path.join(ROOT, "paper_2211_16665_amd", "csrc", "device.hip")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if vals.get("device_source_sha256") != sha or vals.get("kernel") != kernel_tag:
        return None
    return float(vals["traffic_bytes_per_launch"]), vals.get("tiling", "")


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
    (h_ms, e_ms), n_samp = p.kernel_stats()
    bytes_e, edges = algorithmic_bytes_e_forward(nx, ny, nz, w.npml, len(w.freqs), 4, 16,
                                                 int(p.get_option(fw.FWD_OPT_DFT_BLOCK)))
    bytes_b = w.ns * bytes_e - (w.ns - 1) * edges * 4
    bytes_h = w.ns * algorithmic_bytes_h(nx, ny, nz, w.npml, 4)
    del vol
    return {"workload": f"c4_batched window: {nx}x{ny}x{nz}, {w.ns} sources, {len(w.freqs)} freqs, "
                        f"{window} forward + {window} adjoint steps",
            "batched_s": t_batched, "plain_s": t_plain, "speedup": t_plain / t_batched,
            "batched_tuned_s": t_tuned, "speedup_tuned": t_plain / t_tuned, "tuning": tuned,
            "update_e_ms": e_ms, "update_h_ms": h_ms, "samples": n_samp,
            "update_e_bytes_per_launch": bytes_b,
            "update_e_algorithmic_gbs": bytes_b / (e_ms * 1e-3) / 1e9,
            "update_e_frac_of_peak": bytes_b / (e_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "update_h_algorithmic_gbs": bytes_h / (h_ms * 1e-3) / 1e9,
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
                          "update_e": {"fwd_ms": ks[0][0][1], "adj_ms": ks[1][0][1]}}}
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
    bytes_e, _ = algorithmic_bytes_e_forward(nx, ny, nz, w_true.npml, len(w_true.freqs),
                                             tsize, accsize, kb)
    bytes_h = algorithmic_bytes_h(nx, ny, nz, w_true.npml, tsize)
    (h_ms, e_ms), n = ks[0]
    nt = plan.info.nt
    out = {"gradient_s": t, "order2_gradient_s": order2_s, "nt": nt, "dt": plan.info.dt,
           "mcell_per_s": 2.0 * nx * ny * nz * nt / t / 1e6,
           "tiling": {k.lower(): int(plan.get_option(getattr(fw, "FWD_OPT_" + k)))
                      for k in ("BLOCK_X", "BLOCK_Y", "XCD_REMAP", "TILE_ORDER")},
           "update_e_ms": e_ms, "update_h_ms": h_ms, "samples": n,
           "update_e_algorithmic_gbs": bytes_e / (e_ms * 1e-3) / 1e9,
           "update_h_algorithmic_gbs": bytes_h / (h_ms * 1e-3) / 1e9}
    del plan, vol, grad
    torch.cuda.empty_cache()
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


def profile_mode(args, w_true):
    """A short run for hardware-counter collection: one elementwise kernel of
    a known size (256 MiB read + 256 MiB written, the calibration of the byte
    counters), then a forward and an adjoint run of
    ``profile_steps`` steps on the full grid of the workload."""
    import torch
    from paper_2211_16665_amd import fwdem as fw
    n = 256 * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.mul(a, 2.0, out=b)          # one elementwise kernel: 256 MiB read, 256 MiB written
    torch.cuda.synchronize()
    w = w_true.replace(nt=args.profile_steps)
    plan = fw.Plan.from_workload(w, field_dtype=args.field_dtype, acc_mode=args.acc)
    plan.set_option(fw.FWD_OPT_GRAPH_STEPS, 0)
    set_tiling(plan, args.tiling)
    plan.set_model(w.rho)
    plan.basis_build(gamma_rel=1e-12)
    E, vol = plan.forward(want_volume=True)
    plan.adjoint(vol, -E)
    torch.cuda.synchronize()
    print(json.dumps({"profile_steps": args.profile_steps, "copy_bytes": 4 * n,
                      "workload": w.name}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--field-dtype", default="f32")
    ap.add_argument("--acc", default="f64")
    ap.add_argument("--sample-every", type=int, default=2048)
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-vs-plain gradient-time comparison")
    ap.add_argument("--no-td", action="store_true",
                    help="skip the time-domain adjoint study")
    ap.add_argument("--no-vti", action="store_true",
                    help="skip the VTI gradient timing")
    ap.add_argument("--fd-order", type=int, default=2, choices=(2, 4),
                    help="order of the staggered differences of the timed step")
    ap.add_argument("--no-reciprocity", action="store_true",
                    help="skip the towline study of the source-receiver swap")
    ap.add_argument("--no-magnetic", action="store_true",
                    help="skip the gradient step with magnetic receivers")
    ap.add_argument("--no-order4", action="store_true",
                    help="skip the fourth-order gradient timing")
    ap.add_argument("--tiling", default="",
                    help="fixed tiling instead of autotuning: block_x,block_y,xcd_remap,vector")
    ap.add_argument("--profile-workload", default="marine", choices=("marine", "batched"),
                    help="workload of the counter-collection mode")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="counter-collection mode: a 256 MiB device copy (calibration of the "
                         "byte counters) then this many forward and adjoint steps of the "
                         "workload; prints a short JSON line, no metric")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the path has no multi-GPU mode "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2211_16665_amd import fwdem as fw
    from workloads import c2_marine1d

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    w_true = c2_marine1d().replace(fd_order=args.fd_order)
    if args.profile_steps > 0:
        from workloads import c4_batched
        profile_mode(args, c4_batched() if args.profile_workload == "batched" else w_true)
        return
    # background model of the step: the same column without the reservoir
    rho0 = w_true.rho.copy()
    rho0[rho0 == 100.0] = 1.0
    plan = fw.Plan.from_workload(w_true, field_dtype=args.field_dtype, acc_mode=args.acc)
    plan.set_model(w_true.rho)
    d_obs = plan.forward()                               # data of the true model (untimed)
    vol = plan.volume_buffer()
    # tile/schedule autotuning on this workload (untimed setup)
    if args.tiling:
        set_tiling(plan, args.tiling)
        tune_ms = float("nan")
    else:
        tune_ms = plan.autotune(fw.FWD_MODE_FORWARD, vol=vol, steps=32)
    tuned = {k.lower(): int(plan.get_option(getattr(fw, "FWD_OPT_" + k)))
             for k in TILING_KEYS + ("DFT_BLOCK",)}
    tuned["ms_per_forward_step"] = tune_ms
    plan.set_option(fw.FWD_OPT_SAMPLE_EVERY, args.sample_every)
    grad = torch.zeros(plan.shape, dtype=torch.float64, device="cuda")
    stats = {"fwd": [], "adj": []}
    resid_last = []

    def step():
        plan.set_model(rho0)
        plan.basis_build(gamma_rel=1e-12)
        E, _ = plan.forward(vol=vol, want_volume=True)
        stats["fwd"].append(plan.kernel_stats())
        resid = d_obs - E
        resid_last[:] = [resid]
        plan.adjoint(vol, resid, grad=grad)
        stats["adj"].append(plan.kernel_stats())

    for _ in range(args.warmup):
        step()
    stats = {"fwd": [], "adj": []}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    info = plan.info
    nz, ny, nx = plan.shape
    ncells = nx * ny * nz
    nt = info.nt
    updates = 2.0 * plan.ns * ncells * nt * args.steps
    value = updates / elapsed / 1e6

    # roofline of the forward E update (dominant kernel)
    def avg(key, k):
        v = [s[0][k] for s in stats[key] if s[1] > 0]
        n = sum(s[1] for s in stats[key])
        return (float(np.mean(v)) if v else float("nan")), n
    tsize = 4 if args.field_dtype == "f32" else 8
    accsize = 8 if args.acc == "f32" else 16
    kb = int(plan.get_option(fw.FWD_OPT_DFT_BLOCK))
    bytes_e, edges = algorithmic_bytes_e_forward(nx, ny, nz, w_true.npml, len(w_true.freqs),
                                                 tsize, accsize, kb)
    bytes_h = algorithmic_bytes_h(nx, ny, nz, w_true.npml, tsize)
    h_ms = avg("fwd", 0)[0]
    e_ms, n_samp = avg("fwd", 1)
    fused = tuned["schedule"] == 1
    if fused:
        # one launch per step: E and H each read once (no re-read of E by the
        # H update nor of H by the E update)
        n_cells_nodes = (nx + 1) * (ny + 1) * (nz + 1)
        bytes_e = bytes_e + bytes_h - 2 * 3 * n_cells_nodes * tsize
    achieved = bytes_e / (e_ms * 1e-3) / 1e9
    tiling = ",".join(str(tuned[k.lower()]) for k in TILING_KEYS)
    kernel_tag = (f"k_step<float,F64,fwd,{kb}>" if fused else
                  f"k_update_e{'4' if args.fd_order == 4 else ''}<float,F64,fwd,{kb}>")
    mt = measured_traffic(kernel_tag) if args.field_dtype == "f32" and args.acc == "f64" else None
    traffic, traffic_tiling = mt if mt else (None, None)
    kern = {name: {"fwd_ms": avg("fwd", k)[0], "adj_ms": avg("adj", k)[0]}
            for k, name in enumerate(("update_h", "update_e"))}
    if not fused:
        kern["update_h"]["fwd_algorithmic_gbs"] = bytes_h / (h_ms * 1e-3) / 1e9
        kern["update_h"]["bytes_per_launch"] = bytes_h
    kern["update_e"]["fwd_algorithmic_gbs"] = achieved
    out = {
        "metric": "Mcell-updates/s",
        "value": value,
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
        "config": {"workload": "c2_marine1d gradient: 101x101x61 stretched grid (100 m core, "
                               "ratio 1.05), air/0.3 ohm-m water/1 ohm-m sediment/100 ohm-m "
                               "reservoir, 3 freqs 0.25-1.25 Hz, 1 x-dipole, 50 seabed receivers; "
                               "forward + adjoint + gradient"
                               + (", fourth-order differences" if args.fd_order == 4 else ""),
                   "cells": ncells, "nt": nt, "dt": info.dt, "sources": plan.ns,
                   "field_dtype": args.field_dtype, "accumulators": args.acc,
                   "basis_fit": info.basis_fit, "tuning": tuned},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel_tag, "tiling": tiling, "traffic_tiling": traffic_tiling,
                     "bytes_per_launch": bytes_e, "avg_launch_ms": e_ms, "samples": n_samp},
        "kernels_ms": kern,
    }
    if not args.no_td:
        out["adjoint_td"] = adjoint_td_study(plan, resid_last[0], grad, elapsed / args.steps,
                                             w_true.npml)
    if not args.no_vti:                 # changes the plan's model: after the studies above
        out["vti"] = vti_study(plan, w_true, rho0, elapsed / args.steps)
    if not args.no_order4 and args.fd_order == 2:
        out["order4"] = order4_study(w_true, rho0, elapsed / args.steps, tsize, accsize)
    if not args.no_magnetic and args.fd_order == 2 and args.field_dtype == "f32":
        out["magnetic"] = magnetic_study(w_true, rho0, tuned, elapsed / args.steps)
    if not args.no_batched:
        del vol, grad
        torch.cuda.empty_cache()
        out["batched_vs_plain"] = batched_vs_plain()
    if not args.no_reciprocity:
        out["reciprocity"] = reciprocity_study()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w_true)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
