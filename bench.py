"""Benchmark: Mpixel/s to unwrap a synthetic burst-sized interferogram to
within 1e-3 relative L1 of the FP64 oracle's result, on one MI355X.

A step is one complete unwrap (setup, IRLS weight updates, PCG solves with
the cosine-basis preconditioner, mean removal) of one 8192 x 8192 field
(mixed FP16 by default), timed with HIP events from X resident in HBM to U
resident in HBM; the clock stops at the first IRLS iterate whose L1 is
within 1e-3 of the stored oracle value.

Also reported on the same JSON line:
* kernels: every launch of one PCG iteration recorded with HIP events
  inside the first warm-up unwrap, with its algorithmic bytes (HBM-bound
  kernels) or flops (MFMA products); roofline: the dominant one, with HBM
  traffic from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of
  this workload; MFMA products are rated on the flops they execute (the
  folded form: half the dense-equivalent 4NM(N+M) per application);
* hbm_ceilings: measured streaming ceilings of this GPU (the library's own
  copy, read-only and three-read / one-write kernels), against which each
  HBM-bound kernel is also rated;
* mfma_form: the same workload with the folded MFMA preconditioner;
* cg_adaptive / augmented_form: the Section 4.3 schedule and the paper's
  (U, V) form on the same workload;
* precisions: the other plan precisions on the same workload (median of up to 3 unwraps);
* c1, c2, c4: the other configurations (256^2 FP64 against the oracle's U,
  with the oracle timed on one core; 2048^2 plain FP32 under the converged
  schedule against the stored oracle history; 64 uneven tiles batched
  against one FP32 plan per tile);
* cpu_baseline: the FP64 oracle on a bounded sample of the same workload,
  scaled by its recorded iteration counts to the same target.

Other modes (one JSON line each): --batched (64 uneven tiles, batch vs
looped single-tile plans), --paper-shapes (4000 x M), --kernels-only (a
fixed launch sequence for counter runs).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0,
    "bf16": 2500.0, "f16": 2500.0, "f32": 157.3, "f64": 78.6,  # TFLOP/s
}
CONFIGS = {
    "c3": dict(gen="field_c3", N=8192, precision="f16", ref="c3_seed0_8192_float32.json",
               desc="fringe-dense Gaussian-sum phase (+-400 rad), N(0,0.7^2) noise, 2% salt, "
                    "Beta(2,2) weights"),
    "c2": dict(gen="field_c2", N=2048, precision="f32", ref="c2_seed0_2048_float32.json",
               desc="Gaussian-sum phase (+-80 rad), N(0,0.5^2) noise, 3pi step, 64-px "
                    "decorrelated band, Beta(2,2) weights"),
}


def load_reference(name):
    path = os.path.join(ROOT, "oracle", "reference", name)
    with open(path) as fh:
        ref = json.load(fh)
    if not ref.get("complete"):
        raise SystemExit(f"oracle reference {path} is incomplete")
    return ref


def oracle_counts_to_target(ref, target):
    """IRLS index and PCG iterations the oracle needed to reach target."""
    hist = ref["history"]
    pcg = 0
    for k, h in enumerate(hist):
        if h["L1"] <= target:
            return k, pcg
        pcg += h.get("iters", 0)
    return len(hist) - 1, pcg


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(field, ref, target, max_pcg=3):
    """Time the FP64 oracle (as it stands) for one IRLS weight step plus a
    few PCG iterations at full size; scale to the oracle's own counts to the
    target.  Returns the cpu_baseline object."""
    from oracle import reduced as R
    workers = min(16, os.cpu_count() or 1)
    X = field.X.astype(np.float32).astype(np.float64)
    w = field.w.astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    Gv, Gh = R.wrapped_gradients(X)
    N, M = X.shape
    Cv, Ch = R.edge_weights(N, M, w=w)
    U = np.zeros((N, M))
    t1 = time.perf_counter()
    Ov, Oh, b, L1, H = R.weight_step(U, Gv, Gh, Cv, Ch, ref["eps"])
    t2 = time.perf_counter()
    _, info = R.pcg(lambda p: R.apply_A(Ov, Oh, p), lambda r: R.apply_precond(r, workers=workers),
                    b, U, 0.0, max_pcg)
    t3 = time.perf_counter()
    k_t, pcg_t = oracle_counts_to_target(ref, target)
    t_setup, t_weight = t1 - t0, t2 - t1
    t_pcg = (t3 - t2) / max(1, info["iters"])
    est = t_setup + (k_t + 1) * t_weight + pcg_t * t_pcg
    return {
        "value": round(N * M / 1e6 / est, 6), "unit": "Mpixel/s", "cores": workers,
        "kind": "oracle", "nproc": os.cpu_count(), "cpu_model": cpu_model(),
        "cores_note": ("FFT workers capped at 16, the host-CPU share of one GPU on this box "
                       "(numpy's element-wise passes run on one core)"),
        "sample": (f"FP64 oracle on the same {N}x{M} field: setup + 1 IRLS weight step + "
                   f"{info['iters']} PCG iterations timed ({t3 - t0:.1f} s), scaled by the oracle's "
                   f"recorded {k_t} IRLS / {pcg_t} PCG iterations to the same L1 target "
                   f"(est. {est:.0f} s)"),
        "sec_per_pcg_iter": round(t_pcg, 3),
    }


def time_precond(plan, torch, reps=5):
    """Average duration of one preconditioner application (4 GEMM launches)
    with HIP events on the launch stream."""
    r = torch.randn((plan.Np, plan.ld), dtype=plan.dtype, device=plan.device)
    r[plan.N:, :] = 0
    r[:, plan.M:] = 0
    plan.precond(r)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        plan.precond(r)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def time_stencil(plan, torch, reps=20):
    """Average duration of the weighted 5-point operator (plain apply form,
    16 B/px) with HIP events."""
    Ov = torch.rand((plan.Np, plan.ld), dtype=plan.dtype, device=plan.device)
    Oh = torch.rand_like(Ov)
    p = torch.randn_like(Ov)
    plan.operator(Ov, Oh, p)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        plan.operator(Ov, Oh, p)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def kernel_table(launches, prec, form, N, M, flexible):
    """Kernels of one PCG iteration (as recorded inside the unwrap) with
    their time and algorithmic work: bytes per launch for the HBM-bound
    kernels (e = vector element bytes, s = bytes of the fast form's stored
    intermediates), dense-equivalent flops 4NM(N+M) per application for the
    MFMA products."""
    e = 8 if prec == "f64" else 4
    s = 2 if (form == "fast" and prec in ("bf16", "f16")) else e
    px = N * M
    # fast form with plain beta: the last preconditioner pass writes the new
    # direction p (rho from the column pass's spectral sum), the stencil
    # applies the operator only
    spectral = form == "fast" and not flexible
    # fused head: the iterate update d += alpha p rides on the last pass
    # (which reads p for the new direction), not on the fused CG update
    fused = spectral and any(k == "update_dct2" for k, _ in launches)
    bpp = {  # kind -> (kernel, bytes per pixel)
        "stencil": ("stencil_kernel", 4 * e if spectral else 6 * e),  # (z,) p, Ov, Oh in; (p,) q out
        "axpy": ("axpy_kernel", 6 * e),                    # p, q, r, d in; r, d out
        "residual": ("stencil_kernel(residual)", 8 + 5 * e),  # u, d, b, Ov, Oh in; r out
        "rows_dct2": ("fct_rows_fwd_kernel", e + s),        # r in; T1 out
        # CG update fused with the row DCT-II: q, r in; r, T1 out
        "update_dct2": ("fct_rows_fwd_cg_kernel", 3 * e + s),
        "transpose": ("transpose_kernel", 2 * s),
        "cols": ("fct_cols_kernel", 2 * s),
        # T, r, (q) in; z out -- spectral: T, p_old in; p out (fused head:
        # also d in and out)
        "rows_dct3": ("fct_rows_inv_kernel", s + (4 if fused else 3 if flexible else 2) * e),
    }
    n_prod = sum(1 for k, _ in launches if k == "product")
    out = {}
    for kind, ms in launches:
        if kind == "product":
            ent = out.setdefault("gemm_nt_kernel", {"bound": "mfma", "launches": 0, "ms": 0.0,
                                                    "flops_per_launch": 4.0 * px * (N + M) / n_prod,
                                                    "folded": n_prod == 8})
        elif kind in bpp:
            name, b = bpp[kind]
            # the column pass (two FFTs per column in LDS, 4 VALU cycles per
            # wave64 FP32 instruction) is bound by instruction issue; its
            # bytes are listed for reference
            bound = "alu" if kind == "cols" else "hbm"
            ent = out.setdefault(name, {"bound": bound, "launches": 0, "ms": 0.0,
                                        "bytes_per_launch": b * px})
        else:
            ent = out.setdefault(kind, {"bound": "other", "launches": 0, "ms": 0.0})
        ent["launches"] += 1
        ent["ms"] += ms
    for ent in out.values():
        ent["ms"] = round(ent["ms"], 4)
    return out


def profiled_traffic(config, N, prec, form):
    """HBM bytes per launch of each kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary of this workload, if there is one."""
    path = os.path.join(ROOT, "profiles", f"{config}_{N}_{prec}_{form}_hbm_traffic.md")
    out = {}
    if os.path.exists(path):
        with open(path) as fh:
            for line in fh:
                f = line.split()
                if len(f) == 3 and f[0] == "traffic":
                    out[f[1]] = int(f[2])
    return out


# Issue rate of the vector ALUs without packed FP32 (kept out of the code):
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one lane-instruction per lane per
# cycle; a wave64 instruction occupies a 16-lane SIMD for 4 cycles), in
# 10^12 lane-instructions per second.
VALU_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12


def profiled_valu(config, N, prec, form):
    """VALU instructions per launch of each kernel (wave-level count x 64
    lanes) from the committed rocprofv3 SQ_INSTS_VALU summary, if any."""
    path = os.path.join(ROOT, "profiles", f"{config}_{N}_{prec}_{form}_valu.md")
    out = {}
    if os.path.exists(path):
        with open(path) as fh:
            for line in fh:
                f = line.split()
                if len(f) == 3 and f[0] == "valu":
                    out[f[1]] = float(f[2])
    return out


def alu_roofline(kern, valu):
    """Roofline of the kernels bound by instruction issue: lane-instructions
    per second (the profile's VALU count) against VALU_PEAK_T."""
    out = {}
    for name, ent in kern.items():
        if ent["bound"] != "alu" or name not in valu or ent["ms"] <= 0:
            continue
        per_launch = valu[name] * 64.0
        ach = per_launch / (ent["ms"] / ent["launches"] * 1e-3) / 1e12
        out[name] = {"bound": "alu", "achieved": round(ach, 2), "peak": round(VALU_PEAK_T, 2),
                     "unit": "T lane-instructions/s", "frac": round(ach / VALU_PEAK_T, 4),
                     "lane_instructions_per_launch": per_launch}
    return out


def roofline(kern, prec, traffic=None):
    """Roofline object of the dominant kernel (largest time per iteration)
    among those bound by HBM or by MFMA."""
    cand = [(k, v) for k, v in kern.items() if v["bound"] in ("hbm", "mfma")]
    if not cand:
        return None
    name, ent = max(cand, key=lambda kv: kv[1]["ms"])
    ms_launch = ent["ms"] / ent["launches"]
    if ent["bound"] == "mfma":
        # achieved on the flops the products execute: the folded form does
        # half of the dense-equivalent 4NM(N+M) per application
        dense = ent["flops_per_launch"] / (ms_launch * 1e-3) / 1e12
        ex_flops = ent["flops_per_launch"] / (2.0 if ent["folded"] else 1.0)
        ach = ex_flops / (ms_launch * 1e-3) / 1e12
        return {"bound": "mfma", "kernel": name, "achieved": round(ach, 2), "peak": PEAK[prec],
                "unit": "TFLOP/s", "frac": round(ach / PEAK[prec], 4), "traffic": None,
                "flops_per_launch": ex_flops,
                "flops_basis": ("executed: 2NM(N+M) per folded application (half the dense "
                                "products) / launches" if ent["folded"] else
                                "executed: 4NM(N+M) per application / launches"),
                "dense_equivalent_TFLOPs": round(dense, 2),
                "dense_equivalent_frac": round(dense / PEAK[prec], 4),
                "ms_per_launch": round(ms_launch, 4), "launches_per_iter": ent["launches"]}
    ach = ent["bytes_per_launch"] / (ms_launch * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": round(ach, 1), "peak": PEAK["hbm_GBps"],
            "unit": "GB/s", "frac": round(ach / PEAK["hbm_GBps"], 4),
            "traffic": (traffic or {}).get(name),
            "bytes_per_launch": ent["bytes_per_launch"], "ms_per_launch": round(ms_launch, 4),
            "launches_per_iter": ent["launches"]}


def dtype_label(prec, form):
    """Arithmetic of the path: preconditioner / CG vectors / CG scalars."""
    if prec in ("f64", "f32"):
        return prec
    if form == "fast":
        return f"{prec}-storage+f32-transform/f32-vectors/f64-scalars"
    return f"{prec}-mfma/f32-vectors/f64-scalars"


def measure(pkg, torch, N, M, prec, form, X, w, ref, target, a, adaptive=False, steps=None,
            max_irls=None, augmented=False):
    """Warm-up and timed unwraps with one plan form, then the per-kernel
    table of one PCG iteration."""
    t0 = time.perf_counter()
    plan = pkg.Plan(N, M, prec, form=form)
    plan_s = time.perf_counter() - t0
    p = pkg.default_params(prec)
    p.irls_iters = max_irls or a.max_irls
    p.pcg_max = ref["maxit"]
    p.eps = ref["eps"]
    p.l1_target = target
    if adaptive:
        p.cg_schedule = pkg.CG_SCHEDULES["adaptive"]
    p.flexible = a.flexible
    steps = steps or a.steps
    dt = torch.float64 if prec == "f64" else torch.float32
    U = torch.empty((N, M), dtype=dt, device="cuda")
    def run():
        if augmented:
            return plan.unwrap_augmented(X, w, tau=1e-2, delta=1e-6, params=p, stats=True)
        return plan.unwrap(X, w, params=p, out=U, stats=True)

    # per-launch events of one PCG iteration (mid-solve of the second IRLS
    # iteration) recorded inside the first warm-up unwrap
    plan.profile_arm(1, 2 if adaptive else min(50, p.pcg_max - 2))
    for i in range(a.warmup):
        _, st = run()
        if i == 0:
            launches = plan.profile_result()
            plan.profile_arm(-1, -1)
        print(f"[bench] {plan.form} warmup {i}: irls={st['irls_done']} pcg={st['pcg_total']} "
              f"hit={st['target_hit']}", file=sys.stderr, flush=True)
        if i == 0:
            traj = " ".join(f"{h['L1'] / ref['L1_final'] - 1:.2e}"
                            for h in st["history"][:st["irls_done"] + 1])
            print(f"[bench] {plan.form} L1/L1_ref - 1 by IRLS iteration: {traj}", file=sys.stderr,
                  flush=True)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    e0.record(s)
    ev[0].record(s)
    runs = []
    for i in range(steps):
        _, st = run()
        ev[i + 1].record(s)
        runs.append(st)
        print(f"[bench] {plan.form} step {i}: irls={st['irls_done']} pcg={st['pcg_total']} "
              f"hit={st['target_hit']}", file=sys.stderr, flush=True)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    flexible = a.flexible == 1 or (a.flexible < 0 and prec in ("bf16", "f16")
                                   and plan.form != "fast")
    kern = kernel_table(launches, prec, plan.form, N, M, flexible)
    pre = ("stencil", "axpy", "residual")
    return {"plan": plan, "plan_s": plan_s, "form": plan.form, "ms": ms, "step_ms": step_ms,
            "hit": all(r["target_hit"] for r in runs), "last": runs[-1], "kern": kern,
            "roof": roofline(kern, prec, profiled_traffic(a.config, N, prec, plan.form)),
            "iter_ms": round(sum(t for _, t in launches), 4),
            "precond_ms": round(sum(t for k, t in launches if k not in pre), 4)}


def paper_shapes(pkg, torch, synth, a, prec):
    """4000 x M unwraps with the fixed schedule (20 IRLS x 100 PCG): time per
    unwrap with X and w resident in HBM, HIP events, after one warm-up."""
    torch.cuda.set_device(0)
    rows = []
    # the default plan (the mixed-radix fast form at these sides) and the
    # folded MFMA form, unless --form names one
    forms = ["auto", "folded"] if a.form == "auto" else [a.form]
    for M in a.paper_m:
        N = 4000
        f = synth.field_c2(a.seed, N, M)
        X = torch.from_numpy(f.X).to(device="cuda", dtype=torch.float32)
        w = torch.from_numpy(f.w).to(device="cuda", dtype=torch.float32)
        for form in forms:
            print(f"[bench] paper shape {N}x{M} {form}", file=sys.stderr, flush=True)
            plan = pkg.Plan(N, M, prec, form=form)
            p = pkg.default_params(prec)
            p.irls_iters, p.pcg_max = 20, 100
            U = torch.empty((N, M), dtype=torch.float32, device="cuda")
            plan.unwrap(X, w, params=p, out=U)
            s = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(s)
            _, st = plan.unwrap(X, w, params=p, out=U, stats=True)
            e1.record(s)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            rows.append({"N": N, "M": M, "form": plan.form, "ms_per_unwrap": round(ms, 2),
                         "Mpixel_per_s": round(N * M / 1e6 / (ms * 1e-3), 3),
                         "ms_per_pcg_iter": round(ms / max(1, st["pcg_total"]), 4),
                         "pcg_iters": st["pcg_total"], "L1_final": st["L1_final"]})
            plan.close()
            del U
        del X, w
    line = {"metric": "seconds per unwrap of 4000 x M (20 IRLS x 100 PCG)", "unit": "ms",
            "precision": prec, "data": "synthetic (c2-type fields)", "paper_shapes": rows}
    print(json.dumps(line), flush=True)
    return 0


def batched(pkg, torch, synth, a, return_line=False):
    """64 uneven tiles (c1-generator fields, seeds 1000 + t) unwrapped as one
    batch (mixed BF16 and FP32, one grouped launch per PCG phase, PCG
    blocks replayed from captured graphs, launch shapes autotuned per tile
    shape) and one plan per tile in FP32, same schedule (20 IRLS x 100 PCG,
    pcg_rtol 1e-6); HIP events, inputs resident, one warm-up each."""
    torch.cuda.set_device(0)
    shapes = [tuple(int(v) for v in sh) for sh in synth.tile_shapes_c4(0)]
    print(f"[bench] generating {len(shapes)} tiles", file=sys.stderr, flush=True)
    Xs = [torch.from_numpy(synth.field_c4_tile(t, n, m).X).to(device="cuda", dtype=torch.float32)
          for t, (n, m) in enumerate(shapes)]
    px = sum(n * m for n, m in shapes)
    s = torch.cuda.current_stream()

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        out = fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), out

    pb = pkg.default_params("bf16")
    batch = pkg.Batch(shapes, "bf16")
    batch.autotune()
    ms_b, (Ub, stb) = timed(lambda: batch.unwrap(Xs, params=pb, stats=True))
    batch.close()
    p32 = pkg.default_params("f32")
    batch = pkg.Batch(shapes, "f32")
    batch.autotune()
    ms_b32, (Ub32, stb32) = timed(lambda: batch.unwrap(Xs, params=p32, stats=True))
    batch.close()
    n_fast = sum(1 for n, m in shapes if n & (n - 1) == 0 and m & (m - 1) == 0)
    plans = [pkg.Plan(n, m, "f32") for n, m in shapes]
    pf = pkg.default_params("f32")
    ms_l, res = timed(lambda: [pl.unwrap(X, params=pf, stats=True) for pl, X in zip(plans, Xs)])
    forms = sorted({pl.form for pl in plans})
    for pl in plans:
        pl.close()
    edges = [(n - 1) * m + n * (m - 1) for n, m in shapes]
    l1b = [st["L1_final"] / e for st, e in zip(stb, edges)]
    l1l = [r[1]["L1_final"] / e for r, e in zip(res, edges)]
    l1b32 = [st["L1_final"] / e for st, e in zip(stb32, edges)]
    du = max(float((ub - ub.mean() - (r[0] - r[0].mean())).abs().max()) for ub, r in zip(Ub, res))
    du32 = max(float((ub - ub.mean() - (r[0] - r[0].mean())).abs().max())
               for ub, r in zip(Ub32, res))
    line = {"metric": "Mpixel/s, 64 uneven tiles (sides 512..3072) unwrapped, 20 IRLS x 100 PCG",
            "unit": "Mpixel/s", "tiles": len(shapes), "pixels": px,
            "fast_form_tiles": n_fast, "launch_shapes": "autotuned per tile shape",
            "batched": {"precision": "bf16", "value": round(px / 1e6 / (ms_b * 1e-3), 3),
                        "ms": round(ms_b, 1), "pcg_total": sum(st["pcg_total"] for st in stb)},
            "batched_f32": {"precision": "f32", "value": round(px / 1e6 / (ms_b32 * 1e-3), 3),
                            "ms": round(ms_b32, 1),
                            "pcg_total": sum(st["pcg_total"] for st in stb32),
                            "L1_per_edge_max": max(l1b32), "max_abs_U_difference_vs_looped": du32},
            "looped_single_tile": {"precision": "f32", "forms": forms,
                                   "value": round(px / 1e6 / (ms_l * 1e-3), 3),
                                   "ms": round(ms_l, 1),
                                   "pcg_total": sum(r[1]["pcg_total"] for r in res)},
            "speedup": round(ms_l / ms_b, 3),
            "speedup_f32": round(ms_l / ms_b32, 3),
            "equal_accuracy": {"L1_per_edge_max_batched": max(l1b),
                               "L1_per_edge_max_looped": max(l1l),
                               "max_abs_U_difference": du},
            "data": "synthetic (c1-generator tiles)"}
    if return_line:
        return line
    print(json.dumps(line), flush=True)
    return 0


def hbm_ceilings(pkg):
    """Measured streaming ceilings of this GPU (the library's own kernel,
    256 MiB per array, best over the swept grids)."""
    return {k: pkg.stream_probe(k) for k in ("copy", "read", "3r1w")}


def c1_case(pkg, torch, synth, steps=5):
    """Config 1: the 256^2 Gaussian-sum field in FP64, 20 IRLS x <= 100 PCG at
    tolerance 1e-8.  The field meets the Itoh condition (no residues), so U
    is unique up to a constant and is compared pointwise with the oracle's,
    which is timed on one core (threadpoolctl caps every thread pool)."""
    from threadpoolctl import threadpool_limits
    from oracle import reduced as R
    f = synth.field_c1(0, 256, 256)
    X = torch.from_numpy(f.X).to(device="cuda", dtype=torch.float64)
    plan = pkg.Plan(256, 256, "f64")
    p = pkg.default_params("f64")
    p.irls_iters, p.pcg_max, p.pcg_rtol, p.eps = 20, 100, 1e-8, 1e-3
    U = torch.empty((256, 256), dtype=torch.float64, device="cuda")
    plan.unwrap(X, params=p, out=U)
    s = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(s)
    for i in range(steps):
        _, st = plan.unwrap(X, params=p, out=U, stats=True)
        ev[i + 1].record(s)
    torch.cuda.synchronize()
    ms = float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]))
    Ug = U.cpu().numpy()
    plan.close()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        Uo, hist = R.irls(f.X, iters=20, tol=1e-8, maxit=100, eps=1e-3, workers=1)
        t_o = time.perf_counter() - t0
    du = float(np.max(np.abs((Ug - Ug.mean()) - (Uo - Uo.mean()))))
    return {"workload": "c1 seed 0: 256x256 FP64, 8 Gaussians (+-20 rad), ramp, N(0,0.3^2) noise, "
                        "unit weights; 20 IRLS x <= 100 PCG, tol 1e-8",
            "precision": "f64", "ms_per_unwrap": round(ms, 3),
            "value": round(256 * 256 / 1e6 / (ms * 1e-3), 3), "unit": "Mpixel/s",
            "pcg_iters": st["pcg_total"], "L1_final": st["L1_final"],
            "max_abs_U_difference_vs_oracle": du,
            "oracle_1core": {"seconds": round(t_o, 3), "value": round(256 * 256 / 1e6 / t_o, 5),
                             "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
                             "pcg_iters": int(sum(h.get("iters", 0) for h in hist))}}


def c2_case(pkg, torch, synth):
    """Config 2: the 2048^2 field (3 pi step, decorrelated band, Beta(2,2)
    weights) in plain FP32 under the schedule of the stored converged oracle
    reference (every solve to 1e-6): Mpixel/s for the whole schedule and the
    largest relative L1 gap over its iterates (the plain path's bar is
    1e-5)."""
    ref = load_reference("c2_seed0_2048_float32_conv.json")
    n = ref["N"]
    f = synth.field_c2(ref["seed"], n, n)
    X = torch.from_numpy(f.X).to(device="cuda", dtype=torch.float32)
    w = torch.from_numpy(f.w).to(device="cuda", dtype=torch.float32)
    plan = pkg.Plan(n, n, "f32")
    p = pkg.default_params("f32")
    p.irls_iters, p.pcg_max, p.pcg_rtol, p.eps = ref["iters"], ref["maxit"], ref["tol"], ref["eps"]
    U = torch.empty((n, n), dtype=torch.float32, device="cuda")
    plan.unwrap(X, w, params=p, out=U)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    _, st = plan.unwrap(X, w, params=p, out=U, stats=True)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    plan.close()
    gaps = [abs(st["history"][k]["L1"] - ref["history"][k]["L1"]) / ref["history"][k]["L1"]
            for k in range(ref["iters"] + 1)]
    return {"workload": f"c2 seed 0: {n}x{n} plain FP32, {ref['iters']} IRLS, every solve to "
                        f"relres {ref['tol']:g}",
            "precision": "f32", "form": "fast", "ms_per_unwrap": round(ms, 2),
            "value": round(n * n / 1e6 / (ms * 1e-3), 3), "unit": "Mpixel/s",
            "pcg_iters": st["pcg_total"], "oracle_pcg_iters": ref["pcg_total"],
            "max_rel_L1_gap_vs_oracle": max(gaps), "bar": 1e-5, "status": st["status"]}


def kernels_only(pkg, torch, N, M, prec):
    """Fixed launch sequence for counter runs (no unwrap, no oracle)."""
    torch.cuda.set_device(0)
    plan = pkg.Plan(N, M, prec)
    r = torch.randn((plan.Np, plan.ld), dtype=plan.dtype, device=plan.device)
    r[N:, :] = 0
    r[:, M:] = 0
    launches = plan.precond_timed(r, reps=3)
    ms_st = time_stencil(plan, torch, reps=3)   # plain operator form, 16 B/px
    nbytes = 256 << 20
    pkg.stream_probe("copy", nbytes=nbytes, grids=(1024,), reps=3)
    torch.cuda.synchronize()
    out = {"N": N, "M": M, "precision": prec, "form": plan.form,
           "launches": [[k, round(ms, 4)] for k, ms in launches], "stencil_ms": round(ms_st, 4),
           "copy_bytes_each_way": nbytes}
    print(json.dumps(out), flush=True)
    plan.close()
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed unwraps (the median is reported beside the mean)")
    ap.add_argument("--warmup", type=int, default=1, help="at least 1 (it records the kernel table)")
    ap.add_argument("--config", choices=sorted(CONFIGS), default="c3")
    ap.add_argument("--precision", choices=["f64", "f32", "bf16", "f16"], default=None)
    ap.add_argument("--form", choices=["auto", "dense", "folded", "fast"], default="auto",
                    help="preconditioner form of the primary measurement")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--gap", type=float, default=1e-3)
    ap.add_argument("--max-irls", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the streaming-ceiling probes (copy, read, 3 reads + 1 write)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations (c1 256^2 FP64, c2 2048^2 FP32, "
                         "c4 64 uneven tiles)")
    ap.add_argument("--flexible", type=int, choices=[-1, 0, 1], default=-1,
                    help="CG beta: 0 plain, 1 flexible, -1 the plan's default")
    ap.add_argument("--no-precisions", action="store_true",
                    help="skip the other precisions (bf16 / f16 / f32 / f64) on the same workload")
    ap.add_argument("--batched", action="store_true",
                    help="the batched case: 64 uneven tiles (sides 512..3072) in one batch "
                         "against looped single-tile FP32 plans; one JSON line")
    ap.add_argument("--no-augmented", action="store_true",
                    help="skip the measurement of the paper's augmented (U, V) form")
    ap.add_argument("--no-adaptive", action="store_true",
                    help="skip the measurement with the Section 4.3 adaptive CG schedule")
    ap.add_argument("--no-mfma-form", action="store_true",
                    help="skip the second measurement with the MFMA preconditioner")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="4 streaming copies of 256 MiB first (hardware-counter byte calibration)")
    ap.add_argument("--paper-shapes", action="store_true",
                    help="the running-time study of the paper: 4000 x M, M = 2000..16000, "
                         "c2-type fields, fixed 20 x 100 schedule; one JSON line")
    ap.add_argument("--paper-m", type=int, nargs="+", default=[2000, 4000, 8000, 12000, 16000],
                    help="the widths M of --paper-shapes")
    ap.add_argument("--kernels-only", action="store_true",
                    help="a short fixed launch sequence for hardware-counter runs: "
                         "3 preconditioner applications, 3 stencil applications and 4 "
                         "streaming copies of 256 MiB (the byte-count calibration)")
    a = ap.parse_args(argv)
    a.warmup = max(1, a.warmup)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        return 2

    import torch
    import synth
    import paper_2401_09961_amd as pkg

    cfg = CONFIGS[a.config]
    prec = a.precision or cfg["precision"]
    N = M = cfg["N"]
    if a.kernels_only:
        return kernels_only(pkg, torch, N, M, prec)
    if a.copy_calibration:
        # four dispatches of the library's own streaming copy (256 MiB read
        # and written each): the byte calibration of the traffic counters
        torch.cuda.set_device(0)
        pkg.stream_probe("copy", grids=(1024,), reps=3)
        torch.cuda.synchronize()
    if a.paper_shapes:
        return paper_shapes(pkg, torch, synth, a, a.precision or "f16")
    if a.batched:
        return batched(pkg, torch, synth, a)
    ref = load_reference(cfg["ref"])
    L1_ref = ref["L1_final"]
    target = L1_ref * (1.0 + a.gap)
    print(f"[bench] generating {a.config} seed {a.seed} {N}x{M}", file=sys.stderr, flush=True)
    field = getattr(synth, cfg["gen"])(a.seed, N, M)
    dt = torch.float64 if prec == "f64" else torch.float32
    torch.cuda.set_device(0)
    X = torch.from_numpy(field.X).to(device="cuda", dtype=torch.float32).to(dt)
    w = torch.from_numpy(field.w).to(device="cuda", dtype=torch.float32).to(dt)
    primary = measure(pkg, torch, N, M, prec, a.form, X, w, ref, target, a)
    plan = primary["plan"]
    form_primary = plan.form
    # the MFMA route (dense cosine-basis contractions, folded when the sides
    # are even) measured on the same workload when the primary form is not it
    mfma = None
    if plan.form == "fast" and not a.no_mfma_form:
        plan.close()
        form = "folded" if (N % 2 == 0 and M % 2 == 0) else "dense"
        sec = measure(pkg, torch, N, M, prec, form, X, w, ref, target, a,
                      steps=min(max(1, a.steps), 2))
        mfma = {"form": form, "value": round(N * M / 1e6 / (sec["ms"] * 1e-3), 4),
                "ms_per_step": round(sec["ms"], 3), "target_hit": sec["hit"],
                "irls_iters": sec["last"]["irls_done"], "pcg_iters": sec["last"]["pcg_total"],
                "ms_per_pcg_iter": round(sec["ms"] / max(1, sec["last"]["pcg_total"]), 4),
                "roofline": sec["roof"], "precond_ms": sec["precond_ms"]}
        sec["plan"].close()
    # the Section 4.3 adaptive CG schedule on the primary form: time to the
    # same L1 target, or to the IRLS stop of its rule
    adapt = None
    if not a.no_adaptive:
        sec = measure(pkg, torch, N, M, prec, form_primary, X, w, ref, target, a, adaptive=True,
                      steps=1, max_irls=200)
        lst = sec["last"]
        l1 = (lst["history"][lst["irls_done"]]["L1"] if sec["hit"] else lst["L1_final"])
        adapt = {"value": round(N * M / 1e6 / (sec["ms"] * 1e-3), 4),
                 "ms_per_step": round(sec["ms"], 3), "target_hit": sec["hit"],
                 "schedule_stop": lst["schedule_stop"], "irls_iters": lst["irls_done"],
                 "pcg_iters": lst["pcg_total"], "L1_reached": l1,
                 "caps": [h["cap"] for h in lst["history"][:lst["irls_done"]]]}
        sec["plan"].close()
    # the paper's augmented form (U, V^v, V^h), tau = 1e-2, delta = 1e-6, with
    # the primary form's preconditioner on its U block: time and iterations
    # to the same L1 target
    aug = None
    if not a.no_augmented:
        sec = measure(pkg, torch, N, M, prec, form_primary, X, w, ref, target, a, steps=1,
                      augmented=True)
        lst = sec["last"]
        l1 = (lst["history"][lst["irls_done"]]["L1"] if sec["hit"] else lst["L1_final"])
        aug = {"value": round(N * M / 1e6 / (sec["ms"] * 1e-3), 4),
               "ms_per_step": round(sec["ms"], 3), "target_hit": sec["hit"],
               "irls_iters": lst["irls_done"], "pcg_iters": lst["pcg_total"], "L1_reached": l1,
               "ms_per_pcg_iter": round(sec["ms"] / max(1, lst["pcg_total"]), 4),
               "tau": 1e-2, "delta": 1e-6}
        sec["plan"].close()
    # the other precisions on the same workload (the median of as many timed
    # unwraps as the primary measurement, at most 5)
    precs = {}
    if not a.no_precisions:
        for pr in ("bf16", "f16", "f32", "f64"):
            if pr == prec:
                continue
            dtp = torch.float64 if pr == "f64" else torch.float32
            sec = measure(pkg, torch, N, M, pr, "auto", X.to(dtp), w.to(dtp), ref, target, a,
                          steps=min(max(1, a.steps), 3))
            lst = sec["last"]
            med = float(np.median(sec["step_ms"]))
            precs[pr] = {"value": round(N * M / 1e6 / (med * 1e-3), 4),
                         "target_hit": sec["hit"], "irls_iters": lst["irls_done"],
                         "ms_per_pcg_iter": round(med / max(1, lst["pcg_total"]), 4),
                         "steps": len(sec["step_ms"]),
                         "form": sec["form"], "dtype": dtype_label(pr, sec["form"])}
            sec["plan"].close()
    ms, hit, last, roof, kern = (primary["ms"], primary["hit"], primary["last"], primary["roof"],
                                 primary["kern"])
    L1_reached = last["history"][last["irls_done"]]["L1"] if hit else last["L1_final"]
    pcg_per_step = last["pcg_total"]
    form_used = primary["form"]
    line = {
        "metric": "Mpixel/s unwrapped (8192^2 to 1e-3 rel. L1 gap), mixed vs FP64-plain; HBM GB/s",
        "value": round(N * M / 1e6 / (ms * 1e-3), 4),
        "unit": "Mpixel/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms, 3),
        "ms_per_step_median": round(float(np.median(primary["step_ms"])), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype_label(prec, form_used),
        "data": "synthetic",
        "config": {"workload": f"{a.config} seed {a.seed}: {N}x{M} {cfg['desc']}",
                   "precision": prec, "L1_target_rel_gap": a.gap, "L1_ref": L1_ref,
                   "L1_reached": L1_reached, "target_hit": hit,
                   "irls_iters": last["irls_done"], "pcg_iters": pcg_per_step,
                   "ms_per_pcg_iter": round(ms / max(1, pcg_per_step), 4),
                   "plan_create_s": round(primary["plan_s"], 3)},
        "roofline": roof,
        "alu_roofline": alu_roofline(kern, profiled_valu(a.config, N, prec, form_used)),
        "kernels": kern,
        "precond_form": form_used,
        "precond_ms": primary["precond_ms"],
        "iteration_ms_recorded": primary["iter_ms"],
        "mfma_form": mfma,
        "cg_adaptive": adapt,
        "augmented_form": aug,
        "precisions": precs,
    }
    if not a.no_ceilings:
        print("[bench] streaming ceilings", file=sys.stderr, flush=True)
        ceil = hbm_ceilings(pkg)
        line["hbm_ceilings"] = ceil
        if roof and roof["bound"] == "hbm":
            roof["frac_of_measured_copy"] = round(roof["achieved"] / ceil["copy"]["best_GBps"], 4)
            roof["frac_of_measured_3r1w"] = round(roof["achieved"] / ceil["3r1w"]["best_GBps"], 4)
        for name, ent in kern.items():
            if ent["bound"] == "hbm" and ent["ms"] > 0:
                gbs = ent["bytes_per_launch"] * ent["launches"] / (ent["ms"] * 1e-3) / 1e9
                ent["GBps"] = round(gbs, 1)
                ent["frac_of_8TBps"] = round(gbs / PEAK["hbm_GBps"], 4)
                ent["frac_of_measured_3r1w"] = round(gbs / ceil["3r1w"]["best_GBps"], 4)
    if not a.no_configs:
        print("[bench] config 1 (256^2 FP64)", file=sys.stderr, flush=True)
        line["c1"] = c1_case(pkg, torch, synth)
        print("[bench] config 2 (2048^2 FP32, converged schedule)", file=sys.stderr, flush=True)
        line["c2"] = c2_case(pkg, torch, synth)
        print("[bench] config 4 (64 uneven tiles)", file=sys.stderr, flush=True)
        line["c4"] = batched(pkg, torch, synth, a, return_line=True)
    if not a.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(field, ref, target)
    print(json.dumps(line), flush=True)
    if mfma is None:
        plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
