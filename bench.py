#!/usr/bin/env python3
"""Benchmark: forward + adjoint pairs per second on one MI355X.

Workload (default): 2D, Daubechies wavelets with 8 vanishing moments and
boundary correction, M = 2048 x 2048 coefficients, q = 2 (N = 8192 x 8192
Walsh samples), Omega a 12.5 % multilevel variable-density subsample, FP32.
This is the largest configuration of the method measured here; inputs are
synthetic (seeded image-like wavelet coefficients, see tests/inputs.py).

One step = one forward y = P_Omega A x followed by one adjoint A^T P_Omega^T y
of that y, inputs resident in HBM.  The path runs through the C ABI stage by
stage (wh2wav_forward_stage / wh2wav_adjoint_stage, which together are exactly
wh2wav_forward / wh2wav_adjoint).  During warm-up every stage is timed once
with HIP events; in the timed region two events per step bracket the
dominant stage only, on the launch stream, which gives the per-launch
duration used for the roofline.  The line kernels are bound by vector-ALU
issue: their roofline is algorithmic flops (table-product FMAs and FWHT
additions per output sample) against MI355X's published FP32 vector peak,
with this build's issue ceiling (packed FP32 disabled: half that peak) and
the HBM figures alongside.  "pair_hbm" is the whole pair's algorithmic HBM
bytes (minimal-traffic count) over its time, against 8 TB/s.

After the timed region the workload's forward of x and adjoint of a seeded
sample vector are taken in FP32 and FP64; the "cpu_baseline" leg times the
CPU oracle (one whole pair, all cores; a quarter of it on one thread) and
"oracle_check" states every GPU result's relative l2 error against it, and
FP32 against FP64 (also for the small configurations).

More legs are reported in the same JSON line (skip with --no-extras):
* "autograd": the 1024^2 db4 q=1 FP32 operator (25 % Omega) through the
  torch.autograd.Function (gradient of 0.5 ||P A x - y||^2 by backward), the
  plain pair on the same operator, the same gradient captured once as a HIP
  graph and replayed, and 200 FISTA iterations, eager and graph-replayed;
* "round_robin": the default workload on four independent operators in turn
  (about 600 MB live, beyond the 256 MB MALL), pairs/s and the row passes'
  per-launch time and HBM rate;
* "variants": symlets, the periodic extension and the tensor-product basis on
  the roofline workload's shape, 1024^2 db10, 4096^2 db4 (generic line
  kernels), 64^3 db4 and 2048 x 256 db4 (tensor basis);
* "batched": 96 uneven instances (1D 2^12..2^16, 2D 128^2..512^2 and 1024^2,
  db2/db4/db8, q = 1, 2, 10-30 % Omega, FP32) as one graph launch per
  direction (eight branches, largest instances first), against per-instance
  plain calls.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X's published FP32 vector peak (256 CUs x 4 SIMDs x 2.4 GHz, with
# packed FP32 instructions): the roofline's peak.
VALU_PEAK_TFLOPS = 157.3
# The issue ceiling of this build: packed FP32 is disabled, so an FP32 FMA
# retires 16 lanes x 2 flops per SIMD cycle, half the published figure.
VALU_ISSUE_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def stage_bytes(w, m, elem):
    """Algorithmic HBM bytes per launch of each 2D stage (reads + writes, once each)."""
    M, N, Q = 1 << w["j"], 1 << (w["j"] + w["q"]), 1 << w["q"]
    # sample list: a 16-bit natural position per sample and an offset per (row, phase)
    omega_bytes = 0 if m == N * N else 2 * m + 8 * (N * Q + 1)
    return {
        ("fwd", 0): 2 * M * M * elem,                       # x in, B_phi coefficients out
        ("fwd", 1): (M * M + M * N) * elem,                 # column pass: xi in, N x M intermediate out
        ("fwd", 2): (M * N + m) * elem + omega_bytes,       # row pass: intermediate in, y out, sample list
        ("adj", 0): (m + N * M) * elem + omega_bytes,       # row pass: y in, intermediate out
        ("adj", 1): (N * M + M * M) * elem,                 # column pass
        ("adj", 2): 2 * M * M * elem,                       # DWT
    }


def stage_flops(w):
    """Algorithmic flops per launch of the line stages: per output sample of a
    pass, (2nu - 1) FMAs of the table product and log2 M FWHT additions; a
    column pass produces M N samples, a row pass N^2."""
    M, N = 1 << w["j"], 1 << (w["j"] + w["q"])
    per = 2 * (2 * w["nu"] - 1) + w["j"]
    return {("fwd", 1): M * N * per, ("fwd", 2): N * N * per, ("adj", 0): N * N * per, ("adj", 1): M * N * per}


def pair_bytes(w, m, elem):
    """Algorithmic HBM bytes of one forward + adjoint pair by the minimal-traffic
    count: per direction x (s M^2), y (s m), Omega as a bitmask (N^2 / 8) and one
    write plus one read of the M x N intermediate (2 s M N) in 2D."""
    M, N = 1 << w["j"], 1 << (w["j"] + w["q"])
    if w["dim"] == 1:
        return 2 * ((M + m) * elem + (N + 7) // 8)
    return 2 * ((M * M + m) * elem + N * N // 8 + 2 * M * N * elem)


STAGE_NAMES = {("fwd", 0): "idwt", ("fwd", 1): "column_pass_fwd", ("fwd", 2): "row_pass_fwd_gather",
               ("adj", 0): "row_pass_adj_scatter", ("adj", 1): "column_pass_adj", ("adj", 2): "dwt"}
# the kernel each 2D stage launches (the wavelet stages launch one kernel per level)
STAGE_KERNELS = {("fwd", 1): "k_colpass_fwd", ("fwd", 2): "k_rowpass_fwd", ("adj", 0): "k_rowpass_adj",
                 ("adj", 1): "k_colpass_adj"}


def source_digest():
    """Digest of the kernel sources: traffic counters are only valid for the code they measured."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2106_00554_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload):
    """HBM bytes per launch from the committed counter summary, if it matches these sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest() or rec.get("workload") != workload:
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def _rel(a, b):
    import numpy as np
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_oracle_leg(name, X, omega, yv, gpu, small):
    """The CPU oracle on the host cores, and the GPU outputs checked against it.

    The oracle is the separable dense tier: 1D Walsh-coefficient blocks of the
    basis functions (the Walsh matrix times their cell integrals, no fast
    transform), then alpha = sum over bands of A_a X_band A_b^T and the gather.
    One-time construction (boundary functions, blocks) is timed apart.  All
    cores: one whole forward of x and one whole adjoint of yv.  One thread: the
    same pair restricted to a quarter of the Walsh rows n1, times 4.

    gpu holds the GPU outputs of the benchmark workload: forward of x and adjoint
    of yv, in FP32 and FP64.  small holds those of the small configurations.
    """
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import halfline
    from oracle import operator as op
    from tests import inputs

    w = inputs.WORKLOADS[name]
    cfg = op.Config(w["nu"], w["j"], w["q"], w["j0"])
    N = cfg.N
    t0 = time.perf_counter()
    halfline.edge_scaling(cfg.nu, "left"), halfline.edge_scaling(cfg.nu, "right")
    halfline.edge_wavelets(cfg.nu, "left"), halfline.edge_wavelets(cfg.nu, "right")
    t_edges = time.perf_counter() - t0
    t0 = time.perf_counter()
    blocks = op.Blocks2D(cfg)
    t_blocks = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    t0 = time.perf_counter()
    y_ref = op.forward_2d_full(blocks, X, omega)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    x_ref = op.adjoint_2d_full(blocks, yv, omega)
    t_adj = time.perf_counter() - t0
    rows = np.arange(N // 4)
    Y = np.zeros(N * N)
    Y[omega] = yv
    Y_rows = Y.reshape(N, N)[rows].copy()
    del Y
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        op.forward_2d_rows(blocks, X, rows)
        op.adjoint_2d_rows(blocks, Y_rows, rows)
        t_one = 4 * (time.perf_counter() - t0)
    del blocks, Y_rows
    check = {"workload": name,
             "fwd_f32_vs_oracle": _rel(gpu["y32"], y_ref), "adj_f32_vs_oracle": _rel(gpu["x32"], x_ref),
             "fwd_f64_vs_oracle": _rel(gpu["y64"], y_ref), "adj_f64_vs_oracle": _rel(gpu["x64"], x_ref),
             "fwd_f32_vs_f64": _rel(gpu["y32"], gpu["y64"]), "adj_f32_vs_f64": _rel(gpu["x32"], gpu["x64"])}
    small_check = {}
    for key, rec in small.items():
        sw = inputs.WORKLOADS[rec["workload"]]
        scfg = op.Config(sw["nu"], sw["j"], sw["q"], sw["j0"])
        if sw["dim"] == 1:
            A = op.matrix_1d(scfg)
            sy, sx = op.forward_1d(A, rec["x"], rec["omega"]), op.adjoint_1d(A, rec["yv"], rec["omega"])
        else:
            sb = op.Blocks2D(scfg)
            sy, sx = op.forward_2d_full(sb, rec["x"], rec["omega"]), op.adjoint_2d_full(sb, rec["yv"], rec["omega"])
        small_check[key] = {"fwd_vs_oracle": _rel(rec["y"], sy), "adj_vs_oracle": _rel(rec["xa"], sx)}
    for base in {k.rsplit("_", 1)[0] for k in small}:
        if f"{base}_f32" in small and f"{base}_f64" in small:
            a, b = small[f"{base}_f32"], small[f"{base}_f64"]
            small_check[f"{base}_f32"]["fwd_vs_f64"] = _rel(a["y"], b["y"])
            small_check[f"{base}_f32"]["adj_vs_f64"] = _rel(a["xa"], b["xa"])
    check["small_configs"] = small_check
    try:
        host_cpus = len(os.sched_getaffinity(0))
    except AttributeError:
        host_cpus = os.cpu_count() or 1
    baseline = {"value": 1.0 / (t_fwd + t_adj), "unit": "pairs/s", "cores": int(threads), "kind": "oracle",
                "sample": f"one whole forward + adjoint pair of the {name} workload in the separable dense "
                          f"oracle (FP64, BLAS on {threads} threads): forward {t_fwd:.2f} s, adjoint "
                          f"{t_adj:.2f} s; one-time construction apart (boundary functions {t_edges:.1f} s, "
                          f"Walsh-coefficient blocks {t_blocks:.1f} s)",
                "value_1thread": 1.0 / t_one,
                "sample_1thread": f"the same pair restricted to {rows.size} of the {N} Walsh rows n1, on 1 "
                                  f"thread, times {N // rows.size}: {t_one:.1f} s per pair",
                "host_cpus": host_cpus, "cpu_model": _cpu_model(),
                "setup_s": {"boundary_functions": t_edges, "blocks": t_blocks}}
    return baseline, check


def timed(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def autograd_leg(torch, steps):
    from paper_2106_00554_amd import autograd as ag
    from paper_2106_00554_amd.operator import Wh2Wav
    from tests import inputs

    name = "2d_db4_j10_q1_25pct"
    w = inputs.WORKLOADS[name]
    Xt, omega = inputs.workload_inputs(name)
    opr = Wh2Wav(2, w["j"], w["q"], w["nu"], w["j0"], torch.float32, omega)
    xt = torch.tensor(Xt, dtype=torch.float32, device="cuda")
    y0 = opr.forward(xt)
    noise = torch.tensor(inputs.sample_vector(opr.m, 4001), dtype=torch.float32, device="cuda")
    y = y0 + 0.01 * y0.norm() / noise.norm() * noise
    x = torch.zeros(opr.x_shape, dtype=torch.float32, device="cuda", requires_grad=True)
    ybuf = torch.empty_like(y)
    xbuf = torch.empty_like(xt)

    def plain():
        opr.forward(xt, out=ybuf)
        opr.adjoint(ybuf, out=xbuf)

    def grad():
        r = ag.forward(opr, x) - y
        loss = 0.5 * torch.dot(r, r)
        loss.backward()

    for _ in range(3):
        plain()
        grad()
    t_plain = timed(plain, steps, torch)
    t_grad = timed(grad, steps, torch)
    gg = ag.GraphedGradient(opr, y)
    xg = x.detach()
    t_ggrad = timed(lambda: gg(xg), steps, torch)
    lam = 0.01 * float(opr.adjoint(y).abs().max())
    ag.fista(opr, y, lam, 3)  # warm-up
    torch.cuda.synchronize()
    iters = 200
    t0 = time.perf_counter()
    xr = ag.fista(opr, y, lam, iters)
    torch.cuda.synchronize()
    t_fista = time.perf_counter() - t0
    ag.fista_graphed(opr, y, lam, 3)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xg_r = ag.fista_graphed(opr, y, lam, iters)
    torch.cuda.synchronize()
    t_fista_g = time.perf_counter() - t0
    err = float((xr - xt).norm() / xt.norm())
    return {"workload": name, "plain_pairs_per_s": 1.0 / t_plain, "autograd_grads_per_s": 1.0 / t_grad,
            "graphed_grads_per_s": 1.0 / t_ggrad,
            "fista_iters": iters, "fista_iters_per_s": iters / t_fista,
            "fista_graphed_iters_per_s": iters / t_fista_g, "fista_lambda": lam,
            "fista_rel_error_vs_x_true": err,
            "fista_graphed_vs_eager": float((xg_r - xr).norm() / xr.norm())}


def small_configs_leg(torch, steps, outputs=None):
    """The 1D db4 2^10 q=1 workload (FP64 and FP32) and the 2D db4 512^2 q=1 (25 % Omega)
    workload (FP32 and FP64): us per pair and effective GB/s (algorithmic bytes of a pair
    over its time; these working sets fit in the last-level cache, so this is not an HBM
    figure).  If `outputs` is a dict, the forward of x and the adjoint of a seeded sample
    vector are stored there per configuration, for the oracle check."""
    from paper_2106_00554_amd.operator import Wh2Wav
    from tests import inputs

    out = {}
    for name, dtype in (("1d_db4_j10_q1", torch.float64), ("1d_db4_j10_q1", torch.float32),
                        ("2d_db4_j9_q1_25pct", torch.float32), ("2d_db4_j9_q1_25pct", torch.float64)):
        w = inputs.WORKLOADS[name]
        X, omega = inputs.workload_inputs(name)
        opr = Wh2Wav(w["dim"], w["j"], w["q"], w["nu"], w["j0"], dtype, omega)
        x = torch.tensor(X, dtype=dtype, device="cuda")
        y = torch.empty(opr.m, dtype=dtype, device="cuda")
        xa = torch.empty_like(x)

        def pair():
            opr.forward(x, out=y)
            opr.adjoint(y, out=xa)

        for _ in range(5):
            pair()
        t = timed(pair, max(20, steps), torch)
        elem = 8 if dtype == torch.float64 else 4
        M, N = opr.M, opr.N
        if w["dim"] == 1:
            nbytes = 2 * (M + opr.m) * elem
        else:
            nbytes = 2 * (M * M + opr.m + 2 * M * N + 2 * M * M) * elem
        key = f"{name}_{'f64' if elem == 8 else 'f32'}"
        out[key] = {"us_per_pair": t * 1e6, "pairs_per_s": 1.0 / t, "effective_GBs": nbytes / t / 1e9}
        if outputs is not None:
            yv = inputs.sample_vector(opr.m, 41)
            ya = opr.forward(x)
            xb = opr.adjoint(torch.tensor(yv, dtype=dtype, device="cuda"))
            outputs[key] = {"workload": name, "x": X, "omega": omega, "yv": yv,
                            "y": ya.cpu().numpy(), "xa": xb.cpu().numpy()}
    return out


def variants_leg(torch, steps):
    """Pairs/s of the widened operators on the roofline workload's shape and of
    other shapes: symlets, the periodic extension and the tensor-product basis
    at 2048^2 db8 q = 2 (12.5 % Omega), the longest filters at 1024^2 db10
    q = 1 and the generic line kernels (lines beyond the wave kernels) at
    4096^2 db4 q = 1 (10 % Omega), and
    the per-axis path: 64^3 db4 q = 1 (isotropic, 12.5 % Omega) and unequal
    sides 2048 x 256 db4 q = 1 (tensor basis, 12.5 % Omega); all FP32."""
    from paper_2106_00554_amd.operator import Wh2Wav
    from tests import inputs

    name = "2d_db8_j11_q2_12.5pct"
    w = inputs.WORKLOADS[name]
    X, omega = inputs.workload_inputs(name)
    cases = [("sym8", dict(nu=8, j=11, q=2, j0=4, family="sym"), X, omega),
             ("db8_periodic", dict(nu=8, j=11, q=2, j0=4, boundary="per"), X, omega),
             ("db8_tensor", dict(nu=8, j=11, q=2, j0=4, basis2d="tensor"), X, omega)]
    for nu, j, q, j0, dens in ((10, 10, 1, 5, 0.1), (4, 12, 1, 3, 0.1)):
        N = 1 << (j + q)
        cases.append((f"db{nu}_{1 << j}sq" + ("_generic" if j > 11 else ""), dict(nu=nu, j=j, q=q, j0=j0),
                      inputs.coefficients_2d(j, j0, 700 + j), inputs.multilevel_omega_2d(N, dens, 701 + j)))
    cases.append(("db4_64cube_3d", dict(dim=3, nu=4, j=6, q=1, j0=3), inputs.coefficients_nd((64, 64, 64), 760),
                  inputs.uniform_omega(128 ** 3, 0.125, 761)))
    cases.append(("db4_2048x256_tensor", dict(nu=4, j=11, q=1, j0=3, basis2d="tensor", j_axes=(11, 8)),
                  inputs.coefficients_nd((2048, 256), 770), inputs.uniform_omega(4096 * 512, 0.125, 771)))
    out = {}
    for label, kw, Xc, om in cases:
        dim = kw.pop("dim", 2)
        opr = Wh2Wav(dim, kw.pop("j"), kw.pop("q"), kw.pop("nu"), kw.pop("j0"), torch.float32, om, **kw)
        x = torch.tensor(Xc, dtype=torch.float32, device="cuda")
        y = torch.empty(opr.m, dtype=torch.float32, device="cuda")
        xa = torch.empty_like(x)

        def pair():
            opr.forward(x, out=y)
            opr.adjoint(y, out=xa)

        for _ in range(3):
            pair()
        t = timed(pair, max(5, steps // 2), torch)
        out[label] = {"x_shape": list(opr.x_shape), "q": opr.q, "m": opr.m, "us_per_pair": t * 1e6,
                      "pairs_per_s": 1.0 / t}
        del opr, x, y, xa
        torch.cuda.empty_cache()
    return out


def round_robin_leg(torch, steps, name="2d_db8_j11_q2_12.5pct", copies=4):
    """The roofline workload on `copies` independent operators (own plan, sample
    list, workspace and vectors each: about 600 MB live at four copies, more
    than the 256 MB MALL), one pair per step in turn, so that every pass
    reads its inputs from HBM rather than the MALL.  Reports pairs/s and the
    per-launch duration and HBM rate of the two row passes."""
    from paper_2106_00554_amd import _abi
    from paper_2106_00554_amd.operator import Wh2Wav
    from tests import inputs

    w = inputs.WORKLOADS[name]
    X, omega = inputs.workload_inputs(name)
    dt = torch.float32
    ops, xs, ys, xas = [], [], [], []
    for c in range(copies):
        o = Wh2Wav(w["dim"], w["j"], w["q"], w["nu"], w["j0"], dt, omega)
        ops.append(o)
        xs.append(torch.tensor(X * (1.0 + 0.01 * c), dtype=dt, device=o.device))
        ys.append(torch.empty(o.m, dtype=dt, device=o.device))
        xas.append(torch.empty(o.x_shape, dtype=dt, device=o.device))
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    nf = _abi.wh2wav_stage_count(ops[0]._plan, 0)
    na = _abi.wh2wav_stage_count(ops[0]._plan, 1)
    fwd_row, adj_row = ("fwd", nf - 1), ("adj", 0)  # the row passes (gather / scatter)
    keys = [("fwd", s) for s in range(nf)] + [("adj", s) for s in range(na)]

    def run(c, key):
        o, d = ops[c], key[0]
        wsp = o.workspace.data_ptr()
        if d == "fwd":
            _abi.wh2wav_forward_stage(o._plan, key[1], xs[c].data_ptr(), ys[c].data_ptr(), wsp, sp)
        else:
            _abi.wh2wav_adjoint_stage(o._plan, key[1], ys[c].data_ptr(), xas[c].data_ptr(), wsp, sp)

    for c in range(copies):
        for key in keys:
            run(c, key)
    n = steps * copies
    ev = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
          for k in (fwd_row, adj_row)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n):
        c = i % copies
        for key in keys:
            if key in ev:
                ev[key][i][0].record(stream)
                run(c, key)
                ev[key][i][1].record(stream)
            else:
                run(c, key)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    nbytes = stage_bytes(w, ops[0].m, 4)
    out = {"workload": name, "copies": copies, "pairs_per_s": n / elapsed, "ms_per_pair": elapsed / n * 1e3}
    for key, label in ((fwd_row, "k_rowpass_fwd"), (adj_row, "k_rowpass_adj")):
        ms = sum(b.elapsed_time(e) for b, e in ev[key]) / n
        out[label] = {"launch_ms": ms, "hbm_GBs": nbytes[key] / (ms * 1e-3) / 1e9}
    return out


def batched_leg(torch, steps):
    import numpy as np
    from paper_2106_00554_amd.operator import Wh2Wav, Wh2WavBatch
    from tests import inputs

    specs = inputs.batch_specs()
    full = []
    for sp in specs:
        x, omega = inputs.batch_instance(sp)
        full.append((dict(dim=sp["dim"], nu=sp["nu"], j=sp["j"], q=sp["q"], j0=sp["j0"],
                          dtype=torch.float32, omega=omega), x))
    batch = Wh2WavBatch([f for f, _ in full])
    singles = [Wh2Wav(f["dim"], f["j"], f["q"], f["nu"], f["j0"], f["dtype"], f["omega"]) for f, _ in full]
    xs = [torch.tensor(x, dtype=torch.float32, device="cuda") for _, x in full]
    ys = batch.new_outputs(0)
    xa = batch.new_outputs(1)
    # fixed schedule: the autotuner (wh2wav_batch_tune) is kept off the GPU
    # until a host crash seen in one run of it is explained
    batch.set_schedule(8, 1)
    best_ms = None
    sched = batch.schedule()

    def batched():
        batch.forward(xs, ys)
        batch.adjoint(ys, xa)

    def plain():
        for s, x, y, z in zip(singles, xs, ys, xa):
            s.forward(x, out=y)
            s.adjoint(y, out=z)

    batched()
    plain()
    batch.set_mode("fused")
    batched()
    _, in_fused, launches = batch.mode()
    # the two designs in turn, three times each on the same box
    runs = {"branches": [], "fused": []}
    for _ in range(3):
        for mode in ("branches", "fused"):
            batch.set_mode(mode)
            runs[mode].append(timed(batched, steps, torch))
    batch.set_mode("branches")
    t_p = timed(plain, max(1, steps // 2), torch)
    t_b = float(np.median(runs["branches"]))
    t_f = float(np.median(runs["fused"]))
    n = len(specs)
    # algorithmic bytes of one forward + adjoint of every instance: x and y
    # once each, the Omega bitmask, and in 2D one write and one read of the
    # N x M intermediate, per direction
    nbytes = 0
    for f, _ in full:
        M, N = 1 << f["j"], 1 << (f["j"] + f["q"])
        xlen, ntot = (M, N) if f["dim"] == 1 else (M * M, N * N)
        m = ntot if f["omega"] is None else len(f["omega"])
        nbytes += 2 * (4 * xlen + 4 * m + ntot // 8 + (2 * 4 * M * N if f["dim"] == 2 else 0))
    best = min(t_b, t_f)
    # the launch-bound group alone: the 32 2D instances of 128^2 .. 512^2
    small = [k for k, (f, _) in enumerate(full) if f["dim"] == 2 and f["j"] <= 9]
    sb = Wh2WavBatch([full[k][0] for k in small])
    sb.set_schedule(8, 1)
    sxs = [xs[k] for k in small]
    sys_ = sb.new_outputs(0)
    sxa = sb.new_outputs(1)

    def small_batched():
        sb.forward(sxs, sys_)
        sb.adjoint(sys_, sxa)

    small_runs = {"branches": [], "fused": []}
    for mode in ("branches", "fused"):
        sb.set_mode(mode)
        small_batched()
    for _ in range(3):
        for mode in ("branches", "fused"):
            sb.set_mode(mode)
            small_runs[mode].append(timed(small_batched, steps, torch))
    small_out = {"instances": len(small), "fused_launches_per_direction": sb.mode()[2],
                 "runs_ms": {k: [round(v * 1e3, 4) for v in vs] for k, vs in small_runs.items()},
                 "branches_pairs_per_s": len(small) / float(np.median(small_runs["branches"])),
                 "fused_pairs_per_s": len(small) / float(np.median(small_runs["fused"]))}
    sb.close()
    return {"instances": n, "groups": "32 x 1D 2^12..2^16, 32 x 2D 128^2..512^2, 32 x 2D 1024^2",
            "small_group": small_out,
            "pairs_per_s": n / best, "design": "branches" if t_b <= t_f else "fused",
            "branches_pairs_per_s": n / t_b, "fused_pairs_per_s": n / t_f,
            "runs_ms": {k: [round(v * 1e3, 4) for v in vs] for k, vs in runs.items()},
            "fused_instances": in_fused, "fused_launches_per_direction": launches,
            "plain_pairs_per_s": n / t_p, "speedup_vs_plain": t_p / best,
            "ms_per_batch_pair": best * 1e3, "schedule": {"branches": sched[0], "order": sched[1]},
            "algorithmic_bytes_per_pair": nbytes, "hbm_GBs": nbytes / best / 1e9,
            "hbm_frac": nbytes / best / 1e9 / HBM_PEAK_GBS, "tuned_ms": best_ms}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="2d_db8_j11_q2_12.5pct")
    ap.add_argument("--dtype", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--only", choices=["batched", "autograd", "small", "round_robin", "variants"], default=None,
                    help="run one extra leg alone (for profiling) and print its JSON")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="copy MIB MiB device-to-device once before the run (a kernel of known traffic "
                         "for scaling hardware counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the operator is measured on one MI355X only; "
              f"--gpus {args.gpus} is not supported (see the sharding notes in the design document)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.only:
        leg = {"batched": batched_leg, "autograd": autograd_leg, "small": small_configs_leg,
               "round_robin": round_robin_leg, "variants": variants_leg}[args.only]
        print(json.dumps({args.only: leg(torch, max(3, args.steps // 5))}), flush=True)
        return

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

    def run_stage(key):
        d, s = key
        if d == "fwd":
            _abi.wh2wav_forward_stage(opr._plan, s, x.data_ptr(), y.data_ptr(), ws, sp)
        else:
            _abi.wh2wav_adjoint_stage(opr._plan, s, y.data_ptr(), xa.data_ptr(), ws, sp)

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # warm-up; the last warm-up step times every stage to find the dominant one
    for _ in range(max(0, args.warmup - 1)):
        for key in keys:
            run_stage(key)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(keys) + 1)]
    for i, key in enumerate(keys):
        evs[i].record(stream)
        run_stage(key)
    evs[-1].record(stream)
    torch.cuda.synchronize()
    warm_stage = {key: evs[i].elapsed_time(evs[i + 1]) for i, key in enumerate(keys)}
    # the roofline is a single kernel's: in 2D only the line passes launch one
    # kernel per stage (a wavelet stage is one launch per level)
    cands = [k for k in keys if k in STAGE_KERNELS] if w["dim"] == 2 else keys
    dom = max(cands, key=warm_stage.get)

    begin = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    end = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for key in keys:
            if key == dom:
                begin[k].record(stream)
                run_stage(key)
                end[k].record(stream)
            else:
                run_stage(key)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dom_ms = float(np.mean([b.elapsed_time(e) for b, e in zip(begin, end)]))
    nbytes = stage_bytes(w, opr.m, elem)
    achieved = nbytes[dom] / (dom_ms * 1e-3) / 1e9
    kernel = STAGE_KERNELS.get(dom, STAGE_NAMES[dom])
    traffic = traffic_for(kernel, name) if dtype == torch.float32 else None
    flops = stage_flops(w).get(dom)
    if flops is not None and dtype == torch.float32:
        # the line kernels are bound by vector-ALU issue; HBM figures for context
        tflops = flops / (dom_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": kernel, "achieved": tflops, "peak": VALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": tflops / VALU_PEAK_TFLOPS, "traffic": traffic,
                    "algorithmic_flops": flops, "launch_ms": dom_ms,
                    "issue_peak": VALU_ISSUE_TFLOPS, "issue_frac": tflops / VALU_ISSUE_TFLOPS,
                    "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes": nbytes[dom]}}
    else:
        roofline = {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                    "algorithmic_bytes": nbytes[dom], "launch_ms": dom_ms}
    pb = pair_bytes(w, opr.m, elem)
    out = {
        "metric": "forward+adjoint matvec pairs/sec and HBM GB/s (% peak), plain vs batched",
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
        "stages_ms_warmup": {STAGE_NAMES[k]: round(v, 4) for k, v in warm_stage.items()},
        "roofline": roofline,
        "pair_hbm": {"algorithmic_bytes": pb, "achieved_GBs": pb / (elapsed / args.steps) / 1e9,
                     "peak": HBM_PEAK_GBS, "frac": pb / (elapsed / args.steps) / 1e9 / HBM_PEAK_GBS,
                     "path_bytes": sum(nbytes.values()) if w["dim"] == 2 else None},
    }
    # outputs for the oracle check (outside the timed region): forward of x
    # and adjoint of a seeded sample vector, in this precision and the other
    check = {}
    small_out = {} if not args.no_cpu_baseline else None
    if not args.no_cpu_baseline and w["dim"] == 2:
        yv = inputs.sample_vector(opr.m, 31)
        other = torch.float64 if dtype == torch.float32 else torch.float32
        opr2 = Wh2Wav(w["dim"], w["j"], w["q"], w["nu"], w["j0"], other, omega)
        for o, dt in ((opr, dtype), (opr2, other)):
            tag = "32" if dt == torch.float32 else "64"
            check["y" + tag] = o.forward(torch.tensor(X, dtype=dt, device=dev)).cpu().numpy()
            check["x" + tag] = o.adjoint(torch.tensor(yv, dtype=dt, device=dev)).cpu().numpy()
        del opr2
        torch.cuda.empty_cache()
    if not args.no_extras:
        out["autograd"] = autograd_leg(torch, max(5, args.steps // 2))
        out["batched"] = batched_leg(torch, max(3, args.steps // 5))
        out["small_configs"] = small_configs_leg(torch, args.steps, small_out)
        out["round_robin"] = round_robin_leg(torch, max(3, args.steps // 5))
        out["variants"] = variants_leg(torch, args.steps)
    if check:
        out["cpu_baseline"], out["oracle_check"] = cpu_oracle_leg(name, X, omega, yv, check, small_out or {})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
