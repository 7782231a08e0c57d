"""Throughput benchmark of the HGKS stage update on one MI355X.

Workload: 3-D Taylor-Green vortex, 256^3 cells, FP64, smooth mode (linear-weight
WENO5 + smooth gas-kinetic flux), gamma = 1.4, Pr = 0.72, Re = 1600, Ma = 0.1,
CFL 0.4.  One step = one full two-stage update of every cell.  The state is
resident in HBM before the timed region; the timed region is K steps (500 by
default, t = 0.446) in one hgks_step call bracketed by device synchronisations.

Prints one JSON line.  Extra information goes to stderr.

  python bench.py [--steps K] [--warmup W] [--n 256] [--no-cpu]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mcell-updates/s (FP64 vs FP32-form) at stated L2 error; adjoint step time ratio"
UNIT = "Mcell-updates/s"
# The paper's own figure for this workload (TGV 256^3, 64 Xeon E5-2692 cores,
# Sec. 3.2 Table time_table1: 9.09 s per step): context, on other hardware.
PAPER_MCUPS_256 = 256 ** 3 / 9.09 / 1e6

# MI355X published peaks (dense, per GPU)
PEAK_FP64_VECTOR_TFLOPS = 78.6   # 256 CUs x 2.4 GHz x 128 FP64 flop/clk/CU
PEAK_HBM_GBS = 8000.0

# Algorithmic FP64 work of one face in the stage-1 flux kernel, by the scheme's
# own operation count: the moment algebra of the gas-kinetic flux at four Gauss
# points (~1.15k each), the tangential reconstruction to those points (~1.6k)
# and the normal reconstruction with the compatibility state (~0.3k).  This is
# the figure `frac` is priced on.
FLUX_STAGE1_FLOPS_PER_FACE = 6500
# The same face as this library evaluates it, in the closed form of the smooth
# flux (Newtonian stress, Fourier heat flux and the Euler flux Jacobian instead of
# the moment algebra): normal reconstruction + compatibility state + normal
# derivative (639) and tangential reconstruction + four flux evaluations + face
# average (2320), counted as executed FP64 operations (FMA = 2) by rocprofv3 on
# unfused kernels that computed every face once.  Reported as `frac_closed_form`.
FLUX_STAGE1_CLOSED_FORM_FLOPS_PER_FACE = 639 + 2320
# Executed FP64 operations per face of the fused stage-1 kernels as they run
# (halo recomputation included; mean of the three directions, FMA = 2), from
# rocprofv3 SQ_INSTS_VALU_FLOPS_FP64 for the sources with the digest below.
# Reported as `frac_executed`: the share of the FMA peak the kernel issues.
FLUX_STAGE1_EXECUTED_FLOPS_PER_FACE = (2453 + 2371 + 2371) / 3
# Mode Z (WENO-Z reconstruction, full flux integrated over the step): the
# scheme's count per cell-update, about 1e5 FP64 operations over the two stages
# and three directions, i.e. 1e5 / 6 per face and stage.
FLUX_Z_FLOPS_PER_FACE = 1e5 / 6
# HBM bytes per face of the stage-1 flux kernel (mean of the three directions)
# from two rocprofv3 --pmc passes, FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0: the
# factors make the same counters read the known 671 MB in / 671 MB out of the
# library's copy kernel.  Valid only for the kernel sources with this digest
# (profiles/flux_fused_tgv256_kernels.md).
FLUX_STAGE1_HBM_BYTES_PER_FACE = 150.9
FLUX_COUNTERS_SOURCE_DIGEST = "5cb3bf1de8040b20"
# The same counters for the stage-1 FP64 flux of mode Z and of its characteristic
# form at 256^3 (mean of the three directions; profiles/flux_z_isotropic256_kernels.md
# and profiles/flux_zc_shocklet256_kernels.md), per mode: executed FP64 operations
# per face (FMA = 2), HBM bytes per face, and the digest of the sources they hold for.
FLUX_Z_COUNTERS = {
    1: {"executed_flop_per_face": (43299 + 43301 + 43300) / 3, "hbm_bytes_per_face": (549.7 + 647.8 + 600.8) / 3,
        "sources": ("flux_z.hip", "ztile.hpp", "zflux.hpp", "device_common.hpp"), "digest": "de5653f500932ddc"},
    2: {"executed_flop_per_face": (71473 + 71481 + 71475) / 3, "hbm_bytes_per_face": (4040.9 + 4291.0 + 4332.6) / 3,
        "sources": ("flux_zc.hip", "ztile.hpp", "zflux.hpp", "device_common.hpp"), "digest": "fbd92d9b7bf2b700"},
}


def kernel_source_digest(names=("flux_fused.hip", "flux_tile.hpp", "device_common.hpp")):
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2005_08736_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def zflux_roofline(mode: int, faces: int, avg_launch_s: float) -> dict:
    """Roofline of the stage-1 FP64 flux launch of mode Z or its characteristic
    form: priced at the scheme's count per face (frac), and, while the sources are
    those the counters were taken on, at the FP64 operations the kernel issues
    (frac_executed) with its measured HBM traffic."""
    ach = FLUX_Z_FLOPS_PER_FACE * faces / avg_launch_s / 1e12
    out = {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
           "frac": ach / PEAK_FP64_VECTOR_TFLOPS, "flop_per_face": FLUX_Z_FLOPS_PER_FACE,
           "frac_executed": None, "executed_flop_per_face": None, "traffic": None, "hbm_frac": None}
    c = FLUX_Z_COUNTERS.get(mode)
    if c is not None and kernel_source_digest(c["sources"]) == c["digest"]:
        ex = c["executed_flop_per_face"] * faces / avg_launch_s / 1e12
        traffic = c["hbm_bytes_per_face"] * faces
        out.update(frac_executed=ex / PEAK_FP64_VECTOR_TFLOPS, executed_flop_per_face=c["executed_flop_per_face"],
                   traffic=traffic, hbm_frac=traffic / avg_launch_s / 1e9 / PEAK_HBM_GBS)
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(n_cpu: int, steps: int):
    """The oracle as it stands, on the host cores, on a bounded sample of the same
    workload: the Taylor-Green vortex at n_cpu^3 (identical per-cell work)."""
    import oracle
    from paper_2005_08736_amd import cases

    threads = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    p = cases.tgv_params(n_cpu)
    q = cases.tgv_state(n_cpu)
    t0 = time.perf_counter()
    oracle.step(p, q, steps)
    el = time.perf_counter() - t0
    return {
        "value": n_cpu ** 3 * steps / el / 1e6,
        "unit": UNIT,
        "cores": threads,
        "kind": "oracle",
        "sample": f"Taylor-Green {n_cpu}^3, {steps} CFL step(s), FP64, same scheme and per-cell work; {el:.1f} s",
    }


def adjoint_timing(r, reps, torch, label):
    """Time of one step adjoint (hgks_step_vjp, which recomputes the first stage
    itself) at the current state of a run, in that run's arithmetic, and the cost
    of a reverse step under checkpointing (the forward recompute of the step's
    input plus its adjoint) relative to a forward step of the same form."""
    s, q = r["solver"], r["q"]
    dt = float(r["dts"][-1])
    gen = torch.Generator(device=q.device).manual_seed(0)
    lam = torch.randn(q.shape, dtype=q.dtype, device=q.device, generator=gen)
    qn = q.clone()
    s.step_vjp(qn, dt, lam)
    s.profile(True)
    s.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lam = s.step_vjp(qn, dt, lam)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    prof = s.profile_read()
    s.profile(False)
    if not bool(torch.isfinite(lam).all()):
        raise RuntimeError("adjoint produced non-finite values")
    ms_vjp, cnt_vjp = prof["operator_vjp"]
    out = {
        "ms_per_step_vjp": el * 1e3,
        "ms_per_reverse_step_with_recompute": el * 1e3 + r["ms"],
        "ratio_vs_forward_step": (el * 1e3 + r["ms"]) / r["ms"],
        "vjp_only_ratio": el * 1e3 / r["ms"],
        "operator_vjp_avg_launch_ms": ms_vjp / max(cnt_vjp, 1),
        "workload": f"same state and step as the forward run, {label}, dt frozen",
    }
    log(f"[bench] adjoint ({label}): {el * 1e3:.3f} ms per step VJP; reverse step with recompute / forward step = "
        f"{out['ratio_vs_forward_step']:.2f}; operator_vjp {out['operator_vjp_avg_launch_ms']:.3f} ms per launch")
    return out


def adjoint_tgv128_timing(torch, cases, hgks, dev):
    """The adjoint workload itself: gradient of E_k after 100 steps of the 128^3
    Taylor-Green run (plus the seeded 1% solenoidal perturbation) with respect to
    the initial state, checkpoint every 10 steps with recompute, dt frozen from
    the forward run; its wall time against the 100 forward steps alone."""
    from paper_2005_08736_amd import autograd as ag
    n, steps = 128, 100
    p = cases.tgv_params(n)
    q = cases.tgv_state(n)
    U = q[1:4] / q[0] + cases.solenoidal_perturbation(n, seed=0, kmax=4.0, rms=0.01)
    q[4] += 0.5 * q[0] * ((U ** 2).sum(axis=0)) - 0.5 * (q[1:4] ** 2).sum(axis=0) / q[0]
    q[1:4] = q[0] * U
    q0 = torch.from_numpy(q).to(dev)
    dts = ag.cfl_time_steps(p, q0, steps)
    st = ag.Stepper(p, q0)

    def energy(x):
        return 0.5 * torch.sum((x[1] ** 2 + x[2] ** 2 + x[3] ** 2) / x[0]) / x[0].numel()

    # the forward run as the library does it: 100 CFL steps in one call (the same
    # time steps that were frozen above)
    work = q0.clone()
    fwd = hgks.Solver(p, work)
    fwd.step(2)
    work.copy_(q0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fwd.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    e_fwd = energy(work).item()
    fwd.close()
    t0 = time.perf_counter()
    qg = q0.clone().requires_grad_(True)
    J = energy(ag.run_checkpointed(st, qg, dts, every=10))
    J.backward()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    if not bool(torch.isfinite(qg.grad).all()) or abs(J.item() - e_fwd) > 1e-12 * abs(e_fwd):
        raise RuntimeError("adjoint workload: non-finite gradient or a forward pass that differs")
    out = {"workload": "Taylor-Green 128^3 + 1% solenoidal perturbation, dE_k(step 100)/dQ0, checkpoint every 10",
           "s_forward_100_steps": t_fwd, "s_gradient": t_grad, "ratio_gradient_vs_forward": t_grad / t_fwd,
           "note": "gradient = forward pass, then per segment a recompute and the step adjoints, one call per step"}
    log(f"[bench] adjoint workload 128^3 x 100 steps: forward {t_fwd:.3f} s, gradient with checkpointing "
        f"{t_grad:.3f} s, ratio {t_grad / t_fwd:.2f}")
    return out


def adjoint_modez_timing(reps, torch, cases, hgks, dev):
    """The mode-Z adjoint on its checked workload: Taylor-Green 32^3 in mode Z
    (WENO-Z weights and full flux), FP64; forward step time and step-adjoint
    time at the state after 5 CFL steps."""
    n = 32
    p = cases.tgv_params(n, mode=hgks.MODE_WENOZ)
    q = torch.from_numpy(cases.tgv_state(n)).to(dev)
    s = hgks.Solver(p, q)
    dts = s.step(5, return_dt=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(10, dt=float(dts[-1]))
    torch.cuda.synchronize()
    ms_fwd = (time.perf_counter() - t0) / 10 * 1e3
    r = {"solver": s, "q": q, "dts": dts, "ms": ms_fwd}
    out = adjoint_timing(r, reps, torch, "mode Z, Taylor-Green 32^3, FP64")
    out["ms_per_forward_step"] = ms_fwd
    s.close()
    return out


def shocklet_run(args, torch, np, cases, hgks, dev, mode, n=256, ma_t=1.0, seed=0):
    """The shocklet regime of Sec. 3.4: isotropic turbulence at Ma_t = 1.0, 256^3,
    mode Z (conservative or characteristic WENO-Z), args.shocklet_steps CFL steps
    in FP64 (one timed call), then the FP32-flux form along the same time steps
    (one call per step, timed as a whole); Mcell-updates/s of both, the FP32
    form's relative L2 against the FP64 state, or the step at which a form
    reports a non-physical state."""
    steps = args.shocklet_steps
    name = "characteristic" if mode == hgks.MODE_WENOZ_CHAR else "conservative"
    log(f"[bench] isotropic {n}^3 Ma_t {ma_t} seed {seed}, {name} WENO-Z")
    q0 = cases.isotropic_state(n, seed, ma_t)
    p = dict(cases.isotropic_params(n, ma_t, mode=mode))
    N = n ** 3
    out = {"workload": f"isotropic {n}^3, Ma_t {ma_t}, seed {seed}, mode Z with {name} WENO-Z, {steps} CFL steps",
           "steps": steps}
    a = torch.from_numpy(q0).to(dev)
    s = hgks.Solver(p, a)
    s.profile(True)
    s.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        dts = s.step(steps, return_dt=True)
    except hgks.HgksError as e:
        if e.status != hgks.HGKS_E_NONPHYSICAL:
            raise
        out["fp64_nonphysical_at_step"] = s.failed_step()
        log(f"[bench] shocklet run FP64: non-physical state at step {s.failed_step()}")
        s.close()
        return out
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = s.profile_read()
    s.profile(False)
    s.close()
    ms1, c1 = prof["flux_stage1"]
    out["fp64"] = {"value": N * steps / el / 1e6, "unit": UNIT, "ms_per_step": el / steps * 1e3,
                   "dt_first": dts[0], "dt_last": dts[-1], "flux_stage1_avg_launch_ms": ms1 / max(c1, 1),
                   "flux_roofline": zflux_roofline(p["mode"], N, ms1 / max(c1, 1) / 1e3)}
    log(f"[bench] shocklet FP64: {el / steps * 1e3:.2f} ms/step, {out['fp64']['value']:.1f} Mcell-updates/s")
    b = torch.from_numpy(q0).to(dev)
    s32 = hgks.Solver(dict(p, precision=hgks.PREC_F32FLUX), b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, dt in enumerate(dts):
        if s32.step_status(1, dt=float(dt)) != hgks.HGKS_OK:
            out["fp32_nonphysical_at_step"] = i
            log(f"[bench] shocklet run FP32 form: non-physical state at step {i}")
            s32.close()
            return out
    torch.cuda.synchronize()
    el32 = time.perf_counter() - t0
    s32.close()
    A, B = a.cpu().numpy(), b.cpu().numpy()
    mom = float(np.sqrt(np.sum(A[1:4] ** 2)))
    rel = [float(np.linalg.norm(B[k] - A[k])) / (mom if 1 <= k <= 3 else float(np.linalg.norm(A[k])))
           for k in range(5)]
    out["fp32_form"] = {"value": N * steps / el32 / 1e6, "unit": UNIT, "ms_per_step": el32 / steps * 1e3,
                        "rel_l2_vs_fp64_per_field": rel, "rel_l2_vs_fp64": max(rel),
                        "note": "same time steps as the FP64 run, one call per step"}
    log(f"[bench] shocklet FP32 form: {el32 / steps * 1e3:.2f} ms/step, rel L2 vs FP64 {max(rel):.2e}")
    return out


def other_workloads(args, torch, np, cases, hgks, dev):
    """Throughput of the paper's other two workloads, each in its own solver:
    decaying isotropic turbulence at 256^3 (WENO-Z + full flux, mu ~ T^0.76,
    Ma_t = 0.5, seed 0) in FP64 and the FP32-flux form, the same at Ma_t = 1.0
    (the shocklet regime) over a longer run, and the turbulent channel at 128^3
    (walls, tanh mesh, body force; FP64)."""
    out = {}

    def timed(name, p, q0, steps):
        q = torch.from_numpy(q0).to(dev)
        s = hgks.Solver(p, q)
        s.step(2)
        s.profile(True)
        s.profile_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dts = s.step(steps, return_dt=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = s.profile_read()
        s.profile(False)
        ms1, c1 = prof["flux_stage1"]
        n = p["nx"] * p["ny"] * p["nz"]
        r = {"value": n * steps / el / 1e6, "unit": UNIT, "ms_per_step": el / steps * 1e3, "steps": steps,
             "cells": n, "dt": dts[0], "flux_stage1_avg_launch_ms": ms1 / max(c1, 1)}
        if p["mode"] != hgks.MODE_SMOOTH and p.get("precision", hgks.PREC_F64) == hgks.PREC_F64:
            r["flux_roofline"] = zflux_roofline(p["mode"], n, ms1 / max(c1, 1) / 1e3)
        log(f"[bench] {name}: {r['ms_per_step']:.2f} ms/step, {r['value']:.1f} Mcell-updates/s")
        s.close()
        return r, q

    log("[bench] building isotropic 256^3 initial state (Ma_t 0.5, seed 0)")
    qi = cases.isotropic_state(256, 0, 0.5)
    pi = dict(cases.isotropic_params(256, 0.5))
    r64, a = timed("isotropic 256^3 mode Z FP64", pi, qi, args.other_steps)
    pi["precision"] = hgks.PREC_F64
    pi32 = dict(pi)
    pi32["precision"] = hgks.PREC_F32FLUX
    r32, b = timed("isotropic 256^3 mode Z FP32 form", pi32, qi, args.other_steps)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    mom = float(np.sqrt(np.sum(a[1:4] ** 2)))
    rel = max(float(np.linalg.norm(b[k] - a[k])) / (mom if 1 <= k <= 3 else float(np.linalg.norm(a[k])))
              for k in range(5))
    r32["rel_l2_vs_fp64_after_steps"] = rel
    r32["note"] = "each form takes its own CFL steps; the states are compared after the same number of steps"
    out["isotropic_256_modez_fp64"] = r64
    out["isotropic_256_modez_fp32"] = r32
    if args.shocklet_steps > 0:
        out["isotropic_256_modez_ma1"] = shocklet_run(args, torch, np, cases, hgks, dev, hgks.MODE_WENOZ)
        out["isotropic_256_modez_char_ma1"] = shocklet_run(args, torch, np, cases, hgks, dev, hgks.MODE_WENOZ_CHAR)
    pc = dict(cases.channel_params(128, 128, 128))
    rc, _ = timed("channel 128^3 FP64", pc, cases.channel_state(pc, seed=0), 4 * args.other_steps)
    out["channel_128_fp64"] = rc
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500,
                    help="timed Taylor-Green steps per form (500: the 256^3 run the throughput is quoted on)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--cpu-n", type=int, default=128)
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--adjoint-reps", type=int, default=5)
    ap.add_argument("--other-steps", type=int, default=5,
                    help="timed steps of the isotropic (mode Z) and channel workloads (0: skip them)")
    ap.add_argument("--shocklet-steps", type=int, default=100,
                    help="CFL steps of the isotropic Ma_t = 1.0 run (0: skip it)")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2005_08736_amd import cases, hgks

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a ROCm device")
    dev = torch.device("cuda:0")
    n = args.n
    N = n ** 3
    log(f"[bench] building Taylor-Green {n}^3 initial state")
    q_init = cases.tgv_state(n)

    def run(precision):
        p = dict(cases.tgv_params(n))
        p["precision"] = precision
        q = torch.from_numpy(q_init).to(dev)
        s = hgks.Solver(p, q)
        log(f"[bench] precision={precision}: warmup {args.warmup} steps")
        if args.warmup:
            s.step(args.warmup)
        s.profile(True)
        s.profile_read()
        torch.cuda.synchronize()
        log(f"[bench] precision={precision}: timing {args.steps} steps")
        t0 = time.perf_counter()
        dts = s.step(args.steps, return_dt=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = s.profile_read()
        s.profile(False)
        value = N * args.steps / el / 1e6
        log(f"[bench]   {el / args.steps * 1e3:.3f} ms/step, {value:.1f} Mcell-updates/s, dt={dts[0]:.4e}")
        for k, (ms, cnt) in prof.items():
            if cnt:
                log(f"[bench]   {k:12s} {ms:9.3f} ms over {cnt} launches ({ms / cnt:.4f} ms avg)")
        return dict(value=value, ms=el / args.steps * 1e3, prof=prof, dts=dts, solver=s, q=q)

    r64 = run(hgks.PREC_F64)
    adj = adjoint_timing(r64, args.adjoint_reps, torch, "FP64")
    r32 = run(hgks.PREC_F32FLUX)
    adj["fp32_form"] = adjoint_timing(r32, args.adjoint_reps, torch, "FP32-flux form")
    adj["mode_z_32"] = adjoint_modez_timing(args.adjoint_reps, torch, cases, hgks, dev)
    adj["tgv128_gradient"] = adjoint_tgv128_timing(torch, cases, hgks, dev)
    others = other_workloads(args, torch, np, cases, hgks, dev) if args.other_steps > 0 else None
    value = r64["value"]
    ms_per_step = r64["ms"]
    dts = r64["dts"]
    # FP32 form against the FP64 path after the same number of steps
    a, b = r32["q"].cpu().numpy(), r64["q"].cpu().numpy()
    mom = float(np.sqrt(np.sum(b[1:4] ** 2)))
    rel = [float(np.linalg.norm(a[k] - b[k])) / (mom if 1 <= k <= 3 else float(np.linalg.norm(b[k])))
           for k in range(5)]
    fp32 = {"value": r32["value"], "ms_per_step": r32["ms"], "speedup_vs_fp64": r32["value"] / value,
            "rel_l2_vs_fp64_after_steps": max(rel), "rel_l2_per_field": rel,
            "steps_compared": args.warmup + args.steps}
    log(f"[bench] FP32 form: {fp32['speedup_vs_fp64']:.2f}x, rel L2 vs FP64 {max(rel):.2e}")
    prof = r64["prof"]
    ms_flux, cnt_flux = prof["flux_stage1"]
    avg_flux_s = ms_flux / max(cnt_flux, 1) / 1e3
    achieved = FLUX_STAGE1_FLOPS_PER_FACE * N / avg_flux_s / 1e12
    closed = FLUX_STAGE1_CLOSED_FORM_FLOPS_PER_FACE * N / avg_flux_s / 1e12
    counters_current = FLUX_COUNTERS_SOURCE_DIGEST == kernel_source_digest()
    executed = FLUX_STAGE1_EXECUTED_FLOPS_PER_FACE * N / avg_flux_s / 1e12 if counters_current else None
    traffic = FLUX_STAGE1_HBM_BYTES_PER_FACE * N if counters_current else None
    roofline = {
        "bound": "alu",
        "kernel": "flux_fused (stage 1, FP64)",
        "achieved": achieved,
        "peak": PEAK_FP64_VECTOR_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
        "traffic": traffic,
        "avg_launch_ms": avg_flux_s * 1e3,
        "flop_per_face": FLUX_STAGE1_FLOPS_PER_FACE,
        "frac_closed_form": closed / PEAK_FP64_VECTOR_TFLOPS,
        "closed_form_flop_per_face": FLUX_STAGE1_CLOSED_FORM_FLOPS_PER_FACE,
        "frac_executed": executed / PEAK_FP64_VECTOR_TFLOPS if executed is not None else None,
        "executed_flop_per_face": FLUX_STAGE1_EXECUTED_FLOPS_PER_FACE if counters_current else None,
        # the same launch against the HBM roof: measured traffic over the live launch time
        "hbm_achieved_gbs": traffic / avg_flux_s / 1e9 if traffic is not None else None,
        "hbm_frac": traffic / avg_flux_s / 1e9 / PEAK_HBM_GBS if traffic is not None else None,
        "note": "frac prices each face at the scheme's operation count; frac_closed_form at the closed-form "
                "smooth flux this kernel evaluates; frac_executed at the FP64 operations the kernel issues "
                "(rocprofv3 counters); hbm_frac is the measured traffic rate against 8 TB/s",
    }
    d = r64["solver"].diagnostics()
    log(f"[bench] after {args.warmup + args.steps} steps: E_k={d['E_k']:.8f} min_p={d['min_p']:.6f}")
    cpu = None
    if not args.no_cpu:
        log(f"[bench] cpu baseline: oracle on Taylor-Green {args.cpu_n}^3, {args.cpu_steps} step(s)")
        cpu = cpu_baseline(args.cpu_n, args.cpu_steps)
        log(f"[bench] cpu baseline {cpu['value']:.4f} Mcell-updates/s on {cpu['cores']} threads")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": value / cpu["value"] if cpu else None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"taylor_green_{n}^3_fp64_smooth", "cells": N, "cfl": 0.4, "dt": dts[0],
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "fp32_form": fp32,
        "adjoint": adj,
        "other_workloads": others,
        "cpu_baseline": cpu,
        "paper_context": {"value": PAPER_MCUPS_256, "unit": UNIT, "workload": "Taylor-Green 256^3, FP64 (presumed)",
                          "hardware": "64 cores, Intel Xeon E5-2692 2.2 GHz (TianHe-II), MPI",
                          "source": "Sec. 3.2, Table time_table1: 9.09 s per step",
                          "ratio": value / PAPER_MCUPS_256 if n == 256 else None,
                          "note": "another machine's figure: context, not the target"},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
