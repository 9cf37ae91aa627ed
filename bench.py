#!/usr/bin/env python3
"""Benchmark: forward + adjoint pairs per second on one MI355X.

Workload (default): 2D, Daubechies wavelets with 8 vanishing moments and
boundary correction, M = 2048 x 2048 coefficients, q = 2 (N = 8192 x 8192
Walsh samples), Omega a 12.5 % multilevel variable-density subsample, FP32.
This is the HBM-roofline configuration of the method; inputs are synthetic
(seeded image-like wavelet coefficients, see tests/inputs.py).

One step = one forward y = P_Omega A x followed by one adjoint A^T P_Omega^T y
of that y, inputs resident in HBM.  The path runs stage by stage through the
C ABI (wh2wav_forward_stage / wh2wav_adjoint_stage, which together are
exactly wh2wav_forward / wh2wav_adjoint) with HIP events recorded between the
stages on the launch stream, so the per-kernel durations used for the
roofline are measured inside the timed region.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def stage_bytes(w, m, elem):
    """Algorithmic HBM bytes per launch of each 2D stage (reads + writes, once each)."""
    M, N = 1 << w["j"], 1 << (w["j"] + w["q"])
    omega_bytes = (0 if m == N * N else N * N // 8) + 8 * (N + 1)
    return {
        ("fwd", 0): 2 * M * M * elem,                       # x in, B_phi coefficients out
        ("fwd", 1): (M * M + M * N) * elem,                 # column pass: xi in, N x M intermediate out
        ("fwd", 2): (M * N + m) * elem + omega_bytes,       # row pass: intermediate in, y out, Omega mask
        ("adj", 0): (m + N * M) * elem + omega_bytes,       # row pass: y in, intermediate out
        ("adj", 1): (N * M + M * M) * elem,                 # column pass
        ("adj", 2): 2 * M * M * elem,                       # DWT
    }


STAGE_NAMES = {("fwd", 0): "idwt", ("fwd", 1): "column_pass_fwd", ("fwd", 2): "row_pass_fwd_gather",
               ("adj", 0): "row_pass_adj_scatter", ("adj", 1): "column_pass_adj", ("adj", 2): "dwt"}


def cpu_baseline(name, X, omega, budget_s):
    """The oracle (plain sums, no fast transform) on a bounded sample of the workload."""
    import numpy as np
    from oracle import operator as op
    from tests import inputs

    w = inputs.WORKLOADS[name]
    cfg = op.Config(w["nu"], w["j"], w["q"], w["j0"])
    N, M = cfg.N, cfg.M
    rng = np.random.default_rng(0)
    yv = inputs.sample_vector(omega.size, 31)
    op.forward_entries_2d(cfg, X, [0], [0])          # one-time boundary construction, untimed
    nf = 64
    pick = rng.choice(omega.size, nf, replace=False)
    t0 = time.perf_counter()
    op.forward_entries_2d(cfg, X, omega[pick] // N, omega[pick] % N)
    tf = (time.perf_counter() - t0) / nf
    na = 2
    pos = [(M - 1 - int(v), M // 2 + int(v)) for v in rng.integers(0, M // 4, na)]
    t0 = time.perf_counter()
    op.adjoint_entries_2d(cfg, yv, omega, pos)
    ta = (time.perf_counter() - t0) / na
    pair_s = omega.size * tf + M * M * ta
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    return {"value": 1.0 / pair_s, "unit": "pairs/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{nf} forward outputs and {na} adjoint coefficients of the {name} workload, "
                      f"timed one by one; a pair is projected as {omega.size} x and {M * M} x the "
                      f"per-entry times ({tf * 1e3:.2f} ms, {ta:.2f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="2d_db8_j11_q2_12.5pct")
    ap.add_argument("--dtype", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only (the operator is measured on one MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2106_00554_amd import _abi
    from paper_2106_00554_amd.operator import Wh2Wav
    from tests import inputs

    name = args.workload
    w = inputs.WORKLOADS[name]
    dtype = torch.float32 if args.dtype == "fp32" else torch.float64
    elem = 4 if dtype == torch.float32 else 8
    X, omega = inputs.workload_inputs(name)
    opr = Wh2Wav(w["dim"], w["j"], w["q"], w["nu"], w["j0"], dtype, omega)
    dev = opr.device
    x = torch.tensor(X, dtype=dtype, device=dev)
    y = torch.empty(opr.m, dtype=dtype, device=dev)
    xa = torch.empty(opr.x_shape, dtype=dtype, device=dev)
    ws = opr.workspace.data_ptr()
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream
    nf = _abi.wh2wav_stage_count(opr._plan, 0)
    na = _abi.wh2wav_stage_count(opr._plan, 1)
    keys = [("fwd", s) for s in range(nf)] + [("adj", s) for s in range(na)]

    def step(events=None):
        for i, (d, s) in enumerate(keys):
            if events is not None:
                events[i].record(stream)
            if d == "fwd":
                _abi.wh2wav_forward_stage(opr._plan, s, x.data_ptr(), y.data_ptr(), ws, sp)
            else:
                _abi.wh2wav_adjoint_stage(opr._plan, s, y.data_ptr(), xa.data_ptr(), ws, sp)
        if events is not None:
            events[-1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(keys) + 1)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    per_stage = {key: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs])) for i, key in enumerate(keys)}
    nbytes = stage_bytes(w, opr.m, elem)
    dom = max(per_stage, key=per_stage.get)
    achieved = nbytes[dom] / (per_stage[dom] * 1e-3) / 1e9
    out = {
        "metric": "forward+adjoint matvec pairs/sec",
        "value": args.steps / elapsed,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dtype == torch.float32 else "f64",
        "data": "synthetic",
        "config": {"workload": name, "dim": w["dim"], "wavelet": f"db{w['nu']}", "M": 1 << w["j"],
                   "N": 1 << (w["j"] + w["q"]), "q": w["q"], "omega_density": w["density"], "m": opr.m},
        "stages_ms": {STAGE_NAMES.get(k, str(k)): round(v, 4) for k, v in per_stage.items()},
        "roofline": {"bound": "hbm", "kernel": STAGE_NAMES.get(dom, str(dom)), "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(name, X, omega, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
