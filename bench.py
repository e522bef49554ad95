"""Benchmark: refined Schur decompositions per second on one MI355X.

Default workload (the headline line): the precision comparison at n = 4096, the
largest single-GPU configuration. One complex128 matrix A = Q0 T0 Q0^H (Haar Q0,
complex normal eigenvalues at least 1e-3 apart, strictly upper part CN(0,1)/sqrt(n),
seed 2), started from the complex64 Schur basis of complex64(A) (LAPACK cgees).
One step is one complete refinement (Algorithm 4 from the Newton-Schulz start) to
||stril(Q^H A Q)||_F / ||A||_F <= 1e-15 in the FP64 tier (FP32 solve) in one of
three forms of the hp products: native FP64 MFMA ("fp64"), Ozaki INT8 digits for
P = A Q, the start and Q Delta with That and Y native ("ozaki_i8"), or INT8 digits
for every hp product ("ozaki_i8_all"). Every form is run and timed; the line's
value is the fastest form that converges and whose binary128 residual on sampled
rows meets the tolerance, timed over --steps refinements. A, the start and the
workspaces are resident in HBM before timing; each step first restores the start
into Q with a device-to-device copy (inside the timed region).

Other workloads (--workload), each one JSON line of its own:
  single          n = 1024, gaps >= 0.05, cgees start, native FP64 products (also
                  reported as the "n1024" key of the default line);
  precision       the n = 4096 forms plus a product sweep over digit counts;
  batched         2000 matrices, n uniform in [16, 256], each from its own seed
                  with a cgees start, refined together (schur_refine_batched;
                  a step restores all starts with one device copy);
                  matrices/s and the p50 / p99 pass counts;
  dd_continuation A(t_k) = A0 + (k/64) A1, n = 2048, k = 0..63, double-double
                  tier to 1e-28, each step warm-started from the previous one,
                  the first from the zgees Schur form of A0;
  real            the real Schur form of a real n = 2048 matrix (about sqrt(2n/pi)
                  real eigenvalues, conjugate pairs in 2 x 2 blocks, gaps >= 0.05),
                  sgees start, FP64 tier, real FP64 products;
  solvers         the FP32 solve by the tile wavefront and by the recursive block
                  algorithm (Algorithm 3) at n = 1024, 2048, 4096;
  td              the triple-double tier at n = 1024 from a zgees start to 1e-42,
                  checked exactly (Python integers) on sampled rows.

`roofline` covers the dominant kernel of the chosen form, timed with HIP events
on the library's stream during the timed steps: the FP64 GEMM against the FP64
MFMA peak, or the INT8 digit product against the INT8 MFMA peak. `cpu_baseline`
is the binary128 oracle on the host cores: a full refinement at n = 64 timed
as it stands, and binary128 row products at n = 4096 scaled to one refinement.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix peak
INT8_PEAK_TOPS = 5000.0  # MI355X dense INT8 matrix peak
METRIC = "refined Schur decomps/sec to ||stril||/||A||<=1e-15; GEMM % MFMA peak"
TOL = 1e-15


def cpu_baseline(a_big: np.ndarray, q_big: np.ndarray, hp_products: int, rows: int = 16) -> dict:
    """The binary128 oracle as it stands, on the host cores: (1) full refinements of
    the n = 64 configuration (oracle QR start, FP32 solve, binary128 hp), timed;
    (2) binary128 products of `rows` rows of A with Q at the benchmark's n, scaled
    to the hp products of one refinement (the solve and the elementwise work, a few
    percent of a refinement's flops, are not counted there)."""
    import oracle
    import synth

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    g = synth.schur_test_matrix(64, seed=0, gap=0.05)
    z, _ = oracle.schur_qr(g["A"], lp="float")
    reps = 0
    t0 = time.perf_counter()
    while reps < 3 or time.perf_counter() - t0 < 5.0:
        r = oracle.refine(g["A"], z, lp="float", maxit=6, tol=1e-15)
        reps += 1
    t64 = (time.perf_counter() - t0) / reps
    n = a_big.shape[0]
    sel = np.sort(np.random.default_rng(11).choice(n, rows, replace=False))
    qa = oracle.QMat.from_dd(np.asfortranarray(a_big[sel]))
    qq = oracle.QMat.from_dd(q_big)
    t0 = time.perf_counter()
    oracle.gemm(qa, qq)
    dt = time.perf_counter() - t0
    per_refine = dt * (n / rows) * hp_products
    return {"value": 1.0 / per_refine, "unit": "decomps/s", "cores": threads, "kind": "oracle",
            "sample": f"binary128 product of {rows} rows of A with Q at n={n} ({dt:.2f} s), scaled "
                      f"x{n // rows} rows x {hp_products} hp products per refinement (solve and "
                      f"elementwise work not counted); beside it a full oracle refinement at n=64",
            "refinement_n64": {"decomps_per_s": 1.0 / t64, "s_per_refinement": t64,
                               "passes": int(r["iters"]), "status": r["status"], "lp": "float",
                               "hp": "binary128", "reps": reps}}


def pmc_traffic(profile: str, key: str, sources, hash_key: str = "source_sha256_16") -> float | None:
    """Bytes per launch (or per solve) from a committed rocprofv3 PMC summary under
    profiles/, or None when the listed sources have changed since the counters were
    taken (the summary records a hash of them)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", profile)
    csrc = os.path.join(ROOT, "paper_2203_10879_amd", "csrc")
    try:
        text = open(path).read()
        h = hashlib.sha256()
        for f in sources:
            h.update(open(os.path.join(csrc, f), "rb").read())
        vals = dict(line.split(":", 1) for line in text.splitlines()
                    if line.startswith((key + ":", hash_key + ":")))
        if vals[hash_key].split()[0] != h.hexdigest()[:16]:
            return None
        return float(vals[key])
    except (OSError, KeyError, ValueError):
        return None


GEMM_SOURCES = ("gemm.hip", "epilogue.hpp", "kernels.hpp", "common.hpp")
OZAKI_SOURCES = ("ozaki.hip", "ozaki_layout.hpp", "epilogue.hpp", "kernels.hpp", "common.hpp")
CRT_SOURCES = ("crt.hip", "ozaki_layout.hpp", "epilogue.hpp", "kernels.hpp", "common.hpp")
SWEEP_SOURCES = ("trisolve.hip", "trisolve_tiles.inc", "kernels.hpp", "common.hpp")


def base_record(args, value, unit, ms_per_step, dtype, config):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": config}


def single_record(args, n: int, steps: int, warmup: int):
    """One matrix of size n (gaps >= 0.05, seed 1, cgees start), native FP64 tier:
    `steps` timed refinements after `warmup`. Returns the record, the last info, A
    and the start."""
    import torch

    import paper_2203_10879_amd as sr
    import synth

    g = synth.schur_test_matrix(n, seed=1, gap=0.05)
    qh = synth.lp_schur_start(g["A"])
    torch.cuda.set_device(torch.device("cuda:0"))
    A = sr.colmajor(g["A"])
    Q0 = sr.colmajor(qh)
    Q = sr.colmajor_empty(n, n)
    T = sr.colmajor_empty(n, n)
    ws = sr.workspace(n)
    stream = torch.cuda.current_stream()
    kw = dict(compensated=not args.no_compensated, gate=True, workspace=ws, stream=stream)

    def step(timing=False):
        Q.copy_(Q0)
        return sr.schur_refine(A, Q, T, iters=6, tol=TOL, timing=timing, **kw)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(step(timing=True))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = all(i["status"] == "OK" for i in infos)
    ms_gemm = sum(i["ms_hp_gemm"] for i in infos)
    launches = sum(i["hp_gemm_launches"] for i in infos)
    # The roofline covers the full complex products (8 n^3 flop each); the Hermitian
    # products Y = Q^H Q - I form only the tiles on and above the diagonal and are
    # reported beside it.
    herm = sum(i["hp_gemm_herm_launches"] for i in infos)
    ms_herm = sum(i["ms_hp_gemm_herm"] for i in infos)
    full = launches - herm
    avg_gemm_ms = (ms_gemm - ms_herm) / max(1, full)
    achieved = 8.0 * n ** 3 / (avg_gemm_ms * 1e-3) / 1e12
    last = infos[-1]
    out = base_record(args, steps / dt if ok else 0.0, "decomps/s", 1e3 * dt / steps, "f64",
                      {"workload": f"single matrix n={n}, eigenvalue gaps >= 0.05, FP32 cgees start, "
                                   "FP64 tier (FP64 MFMA products, FP32 solve), tol 1e-15",
                       "n": n, "tol": TOL, "compensated": not args.no_compensated,
                       "parallelism": "1 GPU"})
    traffic = (pmc_traffic("refine_n1024_gemm_hbm_traffic.txt", "traffic_bytes_per_launch", GEMM_SOURCES,
                           "gemm_source_sha256_16")
               if n == 1024 else None)
    out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                       "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE x 1.997 + WRITE_SIZE)",
                       "kernel": "complex FP64 GEMM (gemm_kernel<double,...>), full products: 8n^3 flop "
                                 "per launch",
                       "avg_launch_ms": avg_gemm_ms, "launches_per_step": full / steps,
                       "hermitian_products": {"launches_per_step": herm / steps,
                                              "avg_launch_ms": ms_herm / max(1, herm),
                                              "flop_per_launch": 4.0 * n * n * (n + 1)}}
    # The triangular-equation sweep: one solve per update, timed with HIP events around
    # its launches; bytes beyond L2 per solve from the committed counter summary.
    solves = sum(i["updates"] for i in infos)
    ms_solve = sum(i["ms_solve"] for i in infos) / max(1, solves)
    alg_bytes = 12.0 * n * n
    sweep_bytes = (pmc_traffic("trisolve_n1024_hbm_traffic.txt", "sweep_hbm_bytes_per_solve", SWEEP_SOURCES,
                               "trisolve_source_sha256_16")
                   if n == 1024 else None)
    out["sweep"] = {"kernel": "triangular-equation sweep (trisolve_level_kernel<float>, one launch per tile "
                              "diagonal)",
                    "bound": f"latency: {(n + 15) // 16 if n <= 2048 else (n + 31) // 32} dependent launches "
                             "(tile diagonals)",
                    "ms_per_solve": ms_solve, "solves_per_step": solves / steps,
                    "algorithmic_bytes_per_solve": alg_bytes,
                    "algorithmic_GBps": alg_bytes / (ms_solve * 1e-3) / 1e9,
                    "beyond_l2_bytes_per_solve": sweep_bytes,
                    "beyond_l2_GBps": sweep_bytes / (ms_solve * 1e-3) / 1e9 if sweep_bytes else None,
                    "hbm_peak_GBps": 8000.0}
    out.update({"steps": steps, "warmup": warmup, "passes": last["iters"], "hp_gemms": last["hp_gemms"],
                "resid_hist": last["resid_hist"],
                "ms_solve_per_step": sum(i["ms_solve"] for i in infos) / steps,
                "ms_hp_gemm_per_step": ms_gemm / steps, "all_converged": ok})
    return out, last, g["A"], qh


def run_single(args) -> int:
    n = 1024 if args.n is None else args.n
    out, last, a, qh = single_record(args, n, args.steps, args.warmup)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a, qh, hp_products=last["hp_gemms"])
    print(json.dumps(out), flush=True)
    return 0 if out["all_converged"] else 1


HEADLINE_FORMS = ("fp64", "ozaki_i8", "ozaki_i8_all", "ozaki_crt")


def lp_digits_of(args, form: str) -> int:
    """INT8 digits per operand of the lp products in a split form (--lp-digits; the
    native form keeps them in FP32)."""
    return 0 if form == "fp64" else int(args.lp_digits)


def run_default(args) -> int:
    """The headline line: n = 4096, gaps >= 1e-3, every form of the hp products."""
    import torch

    import oracle
    import paper_2203_10879_amd as sr
    import synth

    n = 4096 if args.n is None else args.n
    t0 = time.perf_counter()
    g = synth.schur_test_matrix(n, seed=2, gap=1e-3)
    qh = synth.lp_schur_start(g["A"])
    print(f"# inputs n={n} ready in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.set_device(torch.device("cuda:0"))
    A, Q0 = sr.colmajor(g["A"]), sr.colmajor(qh)
    Q, T = sr.colmajor_empty(n, n), sr.colmajor_empty(n, n)
    form_list = tuple(args.forms.split(",")) if args.forms else HEADLINE_FORMS
    wss = {m: sr.workspace(n, gemm=m, lp_digits=lp_digits_of(args, m)) for m in form_list}
    iters = 8

    def refine(m, timing=False):
        Q.copy_(Q0)
        return sr.schur_refine(A, Q, T, iters=iters, tol=TOL, gemm=m, timing=timing, workspace=wss[m],
                               lp_digits=lp_digits_of(args, m))

    # every form: untimed warmup, then refinements timed one by one with HIP events
    # (the forms interleaved, so that clock drift falls on all alike), then the
    # binary128 residual of its result on sampled rows
    rows = np.sort(np.random.default_rng(7).choice(n, args.rows, replace=False))
    reps = max(2, args.warmup)
    for _ in range(args.warmup):
        for m in form_list:
            refine(m)
    torch.cuda.synchronize()
    ms_each = {m: [] for m in form_list}
    last = {}
    for _ in range(reps):
        for m in form_list:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            last[m] = refine(m)
            e1.record()
            torch.cuda.synchronize()
            ms_each[m].append(e0.elapsed_time(e1))
    forms = {}
    for m in form_list:
        refine(m)
        torch.cuda.synchronize()
        # --rows 0 (profiling runs): no binary128 check, the library's own residual decides
        ev = (oracle.evaluate_rows(g["A"], sr.to_numpy(Q), rows) if args.rows > 0
              else {"stril": float("nan"), "stril_rowmax": float("nan"), "orth": float("nan")})
        inf = last[m]
        meets = inf["status"] == "OK" and (args.rows == 0 or float(ev["stril"]) <= TOL)
        forms[m] = {"status": inf["status"], "passes": inf["iters"], "ms_to_tol": float(np.median(ms_each[m])),
                    "ms_min": float(np.min(ms_each[m])), "resid_hist": inf["resid_hist"],
                    "update_digits": inf["update_slices_hist"] if m != "fp64" else None,
                    "lp_products": (f"INT8, {lp_digits_of(args, m)} digits" if lp_digits_of(args, m)
                                    else "FP32 MFMA"),
                    "quad_stril_rows": float(ev["stril"]), "quad_stril_rowmax": float(ev["stril_rowmax"]),
                    "quad_orth_rows": float(ev["orth"]), "meets_tol": meets}
        print(f"# {m}: {forms[m]['ms_to_tol']:.1f} ms, {inf['iters']} passes, binary128 rows "
              f"{ev['stril']:.2e}", file=sys.stderr, flush=True)
    ok_forms = [m for m in form_list if forms[m]["meets_tol"]]
    if not ok_forms:
        print(json.dumps({"error": "no form met the tolerance", "forms": forms}), flush=True)
        return 1
    best = min(ok_forms, key=lambda m: forms[m]["ms_to_tol"])

    # the timed region: --steps refinements of the chosen form, HIP events around its
    # product and solve launches
    for _ in range(args.warmup):
        refine(best)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(refine(best, timing=True))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = all(i["status"] == "OK" for i in infos)
    steps = args.steps
    out = base_record(args, steps / dt if ok else 0.0, "decomps/s", 1e3 * dt / steps,
                      "f64" if best == "fp64" else "f64+i8",
                      {"workload": f"single matrix n={n}, eigenvalue gaps >= 1e-3 (seed 2), FP32 cgees start, "
                                   f"FP64 tier (FP32 solve), tol 1e-15; hp products as '{best}', the fastest "
                                   "of native FP64 / Ozaki INT8 (P, the start, Q Delta) / Ozaki INT8 (every "
                                   "hp product) / Ozaki scheme II (every hp product) that met the tolerance; "
                                   "the split forms' lp products W^2, W^3, YW from "
                                   f"{args.lp_digits} INT8 digits per operand (native: FP32 MFMA)"
                                   if args.lp_digits else
                                   f"FP64 tier (FP32 solve), tol 1e-15; hp products as '{best}', the fastest "
                                   "of native FP64 / Ozaki INT8 (P, the start, Q Delta) / Ozaki INT8 (every "
                                   "hp product) / Ozaki scheme II (every hp product) that met the tolerance; "
                                   "lp products in FP32 MFMA",
                       "n": n, "tol": TOL, "form": best, "lp_digits": lp_digits_of(args, best),
                       "parallelism": "1 GPU"})
    if best == "fp64":
        ms = sum(i["ms_hp_gemm"] - i["ms_hp_gemm_herm"] for i in infos)
        cnt = sum(i["hp_gemm_launches"] - i["hp_gemm_herm_launches"] for i in infos)
        avg = ms / max(1, cnt)
        achieved = 8.0 * n ** 3 / (avg * 1e-3) / 1e12
        out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": achieved / FP64_PEAK_TFLOPS,
                           "traffic": pmc_traffic("gemm_n4096_hbm_traffic.txt", "traffic_bytes_per_launch",
                                                  GEMM_SOURCES),
                           "kernel": "complex FP64 GEMM (gemm_kernel<double,...>), full products P, That, "
                                     "Q Delta: 8n^3 flop per launch",
                           "avg_launch_ms": avg, "launches_per_step": cnt / steps}
    else:
        ms = sum(i["ms_oz_full"] for i in infos)
        cnt = sum(i["oz_full_launches"] for i in infos)
        pairs = infos[-1]["oz_full_pairs"]
        avg = ms / max(1, cnt)
        achieved = pairs * 8.0 * n ** 3 / (avg * 1e-3) / 1e12
        if best == "ozaki_crt":
            kernel = (f"INT8 residue product (crt_gemm_kernel, Ozaki scheme II, {pairs} moduli), the full "
                      f"products P and That with 55-bit integers: {pairs} x 8n^3 int8 ops per launch")
            traffic = pmc_traffic("crt_gemm_n4096_hbm_traffic.txt", "traffic_bytes_per_launch", CRT_SOURCES)
        else:
            kernel = (f"INT8 digit product (oz_gemm_allpairs_kernel, {pairs} slice pairs), the full products "
                      f"with the main digit count: {pairs} x 8n^3 int8 ops per launch")
            traffic = pmc_traffic("ozaki_allpairs_n4096_hbm_traffic.txt", "traffic_bytes_per_launch",
                                  OZAKI_SOURCES)
        out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                           "frac": achieved / INT8_PEAK_TOPS, "traffic": traffic, "kernel": kernel,
                           "avg_launch_ms": avg, "launches_per_step": cnt / steps,
                           "fp64_equivalent_tflops": 8.0 * n ** 3 / (avg * 1e-3) / 1e12}
    out["roofline"]["traffic_unit"] = ("HBM bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, "
                                       "calibrated on a copy kernel)")
    lastinfo = infos[-1]
    solves = sum(i["updates"] for i in infos)
    out.update({"passes": lastinfo["iters"], "hp_gemms": lastinfo["hp_gemms"], "resid_hist": lastinfo["resid_hist"],
                "ms_hp_products_per_step": sum(i["ms_hp_gemm"] for i in infos) / steps,
                "ms_solve_per_step": sum(i["ms_solve"] for i in infos) / steps,
                "ms_per_solve": sum(i["ms_solve"] for i in infos) / max(1, solves),
                "all_converged": ok, "forms": forms, "quad_rows": args.rows})
    for m in ("ozaki_i8", "ozaki_i8_all", "ozaki_crt"):
        if m in forms and "fp64" in forms:
            out[m + "_speedup_vs_fp64"] = forms["fp64"]["ms_to_tol"] / forms[m]["ms_to_tol"]
    del wss
    torch.cuda.empty_cache()
    if not args.no_secondary:
        # the n = 1024 configuration (native FP64), as a secondary key
        n1024, _, _, _ = single_record(args, 1024, 10, 2)
        out["n1024"] = {k: n1024[k] for k in ("value", "ms_per_step", "passes", "roofline", "sweep",
                                              "resid_hist", "ms_solve_per_step", "ms_hp_gemm_per_step",
                                              "all_converged", "steps")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g["A"], qh, hp_products=lastinfo["hp_gemms"])
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


def run_precision(args) -> int:
    import torch

    import oracle
    import paper_2203_10879_amd as sr
    import synth

    n = 4096 if args.n is None else args.n
    t0 = time.perf_counter()
    g = synth.schur_test_matrix(n, seed=2, gap=1e-3)
    qh = synth.lp_schur_start(g["A"])
    print(f"# inputs n={n} ready in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.set_device(torch.device("cuda:0"))
    A, Q0 = sr.colmajor(g["A"]), sr.colmajor(qh)
    Q, T = sr.colmajor_empty(n, n), sr.colmajor_empty(n, n)
    rows = np.random.default_rng(7).choice(n, args.rows, replace=False)
    # The forms are timed interleaved (one refinement of each per step, each timed
    # with HIP events on the current stream), so that clock drift over the run falls
    # on all of them alike.
    modes = HEADLINE_FORMS
    wss = {m: sr.workspace(n, gemm=m, lp_digits=lp_digits_of(args, m)) for m in modes}
    for _ in range(args.warmup):
        for m in modes:
            Q.copy_(Q0)
            sr.schur_refine(A, Q, T, iters=8, tol=TOL, gemm=m, workspace=wss[m], lp_digits=lp_digits_of(args, m))
    torch.cuda.synchronize()
    infos = {m: [] for m in modes}
    ms_each = {m: [] for m in modes}
    for _ in range(args.steps):
        for m in modes:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            Q.copy_(Q0)
            infos[m].append(sr.schur_refine(A, Q, T, iters=8, tol=TOL, gemm=m, timing=True, workspace=wss[m],
                                            lp_digits=lp_digits_of(args, m)))
            e1.record()
            torch.cuda.synchronize()
            ms_each[m].append(e0.elapsed_time(e1))
    forms = {}
    for m in modes:
        Q.copy_(Q0)
        sr.schur_refine(A, Q, T, iters=8, tol=TOL, gemm=m, workspace=wss[m], lp_digits=lp_digits_of(args, m))
        torch.cuda.synchronize()
        ev = oracle.evaluate_rows(g["A"], sr.to_numpy(Q), rows)
        inf, last = infos[m], infos[m][-1]
        launches = sum(i["hp_gemm_launches"] for i in inf)
        forms[m] = {"status": last["status"], "passes": last["iters"],
                    "ms_to_tol": float(np.median(ms_each[m])), "ms_min": float(np.min(ms_each[m])),
                    "ms_hp_products": sum(i["ms_hp_gemm"] for i in inf) / args.steps,
                    "avg_hp_product_ms": sum(i["ms_hp_gemm"] for i in inf) / max(1, launches),
                    "ms_solve": sum(i["ms_solve"] for i in inf) / args.steps,
                    "resid_hist": last["resid_hist"], "update_digits": last["update_slices_hist"],
                    "quad_stril_rows": float(ev["stril"]), "quad_orth_rows": float(ev["orth"])}
        print(f"# {m}: {forms[m]['ms_to_tol']:.1f} ms (median of {args.steps})", file=sys.stderr, flush=True)
    del wss
    # The product P = A Q-hat per form: Ozaki INT8 with s digits per operand (pairs up
    # to s + t = s + 1, splits included) and native FP64, timed with HIP events and
    # compared with the binary128 product on 8 of the sampled rows.
    rows8 = np.sort(rows[:8])
    ref_hi, ref_lo = oracle.gemm(np.asfortranarray(g["A"][rows8]), qh).to_dd()
    scale = float(np.linalg.norm(ref_hi))
    P = sr.colmajor_empty(n, n)
    idx = torch.as_tensor(rows8, device="cuda")

    def rel_err():
        p = P.index_select(0, idx).cpu().numpy()
        return float(np.linalg.norm((p - ref_hi) - ref_lo) / scale)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ws_oz = torch.empty(int(sr.lib().sr_ozaki_ws_bytes(n, n, n, 8, 8)), dtype=torch.uint8, device="cuda")
    sweep = []
    for sd in (3, 4, 5, 6, 7, 8):
        ms = timed(lambda: sr.sr_ozaki_zgemm(A, Q0, P, slices_a=sd, slices_b=sd, dmax=sd + 1, ws=ws_oz))
        pairs = sd * (sd + 1) // 2
        sweep.append({"form": f"int8 s={sd}", "pairs": pairs, "ms": ms, "rel_err_rows": rel_err(),
                      "int8_frac_of_peak": pairs * 8.0 * n ** 3 / (ms * 1e-3) / (INT8_PEAK_TOPS * 1e12)})
    del ws_oz
    ws_crt = torch.empty(int(sr.lib().sr_crt_ws_bytes(n, n, n, 55)), dtype=torch.uint8, device="cuda")
    for bits in (23, 31, 39, 47, 55):
        ms = timed(lambda: sr.sr_crt_zgemm(A, Q0, P, bits=bits, ws=ws_crt))
        nm = int(sr.lib().sr_crt_moduli(n, bits))
        sweep.append({"form": f"crt bits={bits}", "moduli": nm, "ms": ms, "rel_err_rows": rel_err(),
                      "int8_frac_of_peak": nm * 8.0 * n ** 3 / (ms * 1e-3) / (INT8_PEAK_TOPS * 1e12)})
    del ws_crt
    for comp in (False, True):
        ms = timed(lambda: sr.sr_zgemm(A, Q0, P, compensated=comp))
        sweep.append({"form": "fp64" + (" compensated" if comp else ""), "ms": ms, "rel_err_rows": rel_err(),
                      "fp64_frac_of_peak": 8.0 * n ** 3 / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS})
    print("# product sweep: " + ", ".join(f"{r['form']} {r['ms']:.2f} ms {r['rel_err_rows']:.1e}" for r in sweep),
          file=sys.stderr, flush=True)
    oz, fp = forms["ozaki_i8"], forms["fp64"]
    ok = oz["status"] == "OK" and fp["status"] == "OK"
    out = base_record(args, 1e3 / oz["ms_to_tol"] if ok else 0.0, "decomps/s", oz["ms_to_tol"], "f64+i8",
                      {"workload": f"precision comparison n={n}, eigenvalue gaps >= 1e-3, FP32 cgees start; "
                                   "value = Ozaki INT8 form (P = AQ, the start's products and Q Delta on "
                                   "INT8 digits; That and Y native FP64); ozaki_i8_all: every hp product "
                                   "from INT8 digits",
                       "n": n, "tol": TOL, "quad_rows": args.rows})
    out["forms"] = forms
    out["ozaki_speedup_vs_fp64"] = fp["ms_to_tol"] / oz["ms_to_tol"]
    out["ozaki_all_speedup_vs_fp64"] = fp["ms_to_tol"] / forms["ozaki_i8_all"]["ms_to_tol"]
    out["ozaki_crt_speedup_vs_fp64"] = fp["ms_to_tol"] / forms["ozaki_crt"]["ms_to_tol"]
    out["product_sweep"] = {"product": f"P = A Q-hat, n={n}", "error": "relative Frobenius error on 8 rows "
                            "against the binary128 product", "forms": sweep}
    # the value's form: its full INT8 products P = A Q (HIP events on the library's stream)
    inf = infos["ozaki_i8"]
    cnt = sum(i["oz_full_launches"] for i in inf)
    avg = sum(i["ms_oz_full"] for i in inf) / max(1, cnt)
    npairs = inf[-1]["oz_full_pairs"]
    achieved = npairs * 8.0 * n ** 3 / (avg * 1e-3) / 1e12 if avg > 0 else 0.0
    out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                       "frac": achieved / INT8_PEAK_TOPS,
                       "traffic": pmc_traffic(f"ozaki_allpairs_n{n}_hbm_traffic.txt", "traffic_bytes_per_launch",
                                              OZAKI_SOURCES),
                       "traffic_unit": ("HBM bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, "
                                        "calibrated on a copy kernel)"),
                       "kernel": f"all-pairs INT8 product (oz_gemm_allpairs_kernel<0, S>) P = A Q, {npairs} digit "
                                 f"pairs x 8 n^3 ops per launch",
                       "avg_launch_ms": avg, "launches_per_step": cnt / args.steps}
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


def run_batched(args) -> int:
    import synth

    count = args.count
    sizes = [int(x) for x in synth.batched_sizes(count, seed=3)]
    t0 = time.perf_counter()
    # inputs are made before the GPU is touched
    data = synth.batched_inputs(sizes, 10000, workers=min(16, os.cpu_count() or 1))
    print(f"# {count} inputs ready in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    import torch

    import oracle
    import paper_2203_10879_amd as sr

    torch.cuda.set_device(torch.device("cuda:0"))
    As = [sr.colmajor(a) for a, _ in data]
    # the starts and the refined Q of all matrices are column-major views into one
    # buffer each, so that a step restores every start with a single copy
    offs = np.concatenate([[0], np.cumsum([n * n for n in sizes])]).astype(np.int64)
    q0_flat = torch.empty(int(offs[-1]), dtype=torch.complex128, device="cuda")
    q_flat = torch.empty_like(q0_flat)

    def view(flat, i):
        n = sizes[i]
        return flat[int(offs[i]):int(offs[i + 1])].view(n, n).T

    for i, (_, q) in enumerate(data):
        view(q0_flat, i).copy_(sr.colmajor(q))
    Qs = [view(q_flat, i) for i in range(count)]
    Ts = [sr.colmajor_empty(n, n) for n in sizes]
    ws = sr.workspace_batched(sizes)

    def step():
        q_flat.copy_(q0_flat)
        return sr.schur_refine_batched(As, Qs, Ts, iters=8, tol=TOL, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        rc, infos = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) / args.steps
    passes = np.array([i["iters"] for i in infos])
    ok = rc == 0
    # binary128 check of a few matrices
    checks = []
    for i in np.random.default_rng(5).choice(count, 4, replace=False):
        ev = oracle.evaluate(data[i][0], sr.to_numpy(Qs[i]), sr.to_numpy(Ts[i]))
        checks.append({"n": sizes[i], "stril": float(ev["stril"]), "orth": float(ev["orth"])})
    flops = sum(8.0 * n ** 3 * inf["hp_gemms"] for n, inf in zip(sizes, infos))
    out = base_record(args, count / dt if ok else 0.0, "decomps/s", 1e3 * dt, "f64",
                      {"workload": f"batched: {count} matrices, n uniform in [16, 256] (seed 3), "
                                   "eigenvalue gaps >= 0.05, FP32 cgees starts, FP64 tier, tol 1e-15, "
                                   "one schur_refine_batched call per step",
                       "count": count, "tol": TOL,
                       "tile_edges": {str(b): sr.lib().sr_batched_tile_edge(b) for b in (32, 64, 128, 192, 256)},
                       "blocks_per_cu": {str(b): sr.lib().sr_batched_tile_grid(b) for b in (32, 64, 128, 192, 256)}})
    out.update({"passes_p50": float(np.percentile(passes, 50)), "passes_p99": float(np.percentile(passes, 99)),
                "passes_max": int(passes.max()), "hp_flops_per_step": flops,
                "hp_tflops_effective": flops / dt / 1e12, "quad_checks": checks})
    # The products run inside one HIP graph per call, so no launch can be timed on its
    # own: the figure is the whole step's hp flops (8 n^3 per product; the Hermitian Y
    # counted in full though it forms the tiles on and above the diagonal only) over
    # the step's time, a lower bound on the rate of the grouped products.
    out["roofline"] = {"bound": "mfma", "achieved": flops / dt / 1e12, "peak": FP64_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": flops / dt / 1e12 / FP64_PEAK_TFLOPS, "traffic": None,
                       "kernel": "grouped complex FP64 products of all matrices (gemm_grouped_kernel<double,...>)",
                       "scope": "whole step (solves, elementwise work and the graph's gaps included)"}
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


def run_dd_continuation(args) -> int:
    import torch

    import oracle
    import paper_2203_10879_amd as sr
    import synth

    n = 2048 if args.n is None else args.n
    steps = args.cont_steps
    t0 = time.perf_counter()
    g = synth.schur_test_matrix(n, seed=4, gap=0.05)
    a1 = synth.continuation_perturbation(n, seed=5)
    q0 = synth.hp_schur_start(g["A"])
    pairs = [synth.continuation_step_dd(g["A"], a1, k) for k in range(steps)]
    print(f"# inputs n={n} ready in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.set_device(torch.device("cuda:0"))
    dev = [(sr.colmajor(h), sr.colmajor(l)) for h, l in pairs]
    Qh, Ql = sr.colmajor(q0), sr.colmajor(np.zeros_like(q0))
    Th, Tl = sr.colmajor_empty(n, n), sr.colmajor_empty(n, n)
    ws = sr.workspace_dd(n, update_slices=-1)
    per = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(steps):
        info = sr.schur_refine_dd(dev[k][0], dev[k][1], Qh, Ql, Th, Tl, iters=8, tol=1e-28, timing=True,
                                  workspace=ws, update_slices=-1)
        per.append({"k": k, "status": info["status"], "passes": info["iters"], "ms": info["ms_total"],
                    "ms_hp": info["ms_hp_gemm"], "resid": info["resid"], "ms_full": info["ms_oz_full"],
                    "full": info["oz_full_launches"], "pairs": info["oz_full_pairs"]})
        if k % 8 == 0:
            print(f"# step {k}: {info['status']} {info['iters']} passes {info['ms_total']:.1f} ms",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    ok = all(p["status"] == "OK" for p in per)
    rows = np.random.default_rng(9).choice(n, args.rows, replace=False)
    ah, al = pairs[-1]
    ev = oracle.evaluate_rows(oracle.QMat.from_dd(ah, al),
                              oracle.QMat.from_dd(sr.to_numpy(Qh), sr.to_numpy(Ql)), rows)
    hp_ms = sum(p["ms_hp"] for p in per)
    # the product launches P = A Q and That alone (HIP events on the library's stream)
    cnt = sum(p["full"] for p in per)
    avg = sum(p["ms_full"] for p in per) / max(1, cnt)
    npairs = per[-1]["pairs"]
    achieved = npairs * 8.0 * n ** 3 / (avg * 1e-3) / 1e12 if avg > 0 else 0.0
    out = base_record(args, steps / dt if ok else 0.0, "decomps/s", 1e3 * dt / steps, "dd(int8)",
                      {"workload": f"double-double continuation A0 + (k/{steps}) A1, n={n}, A1 = 1e-3 CN(0,1) "
                                   "(46-bit), tol 1e-28, warm starts, first from zgees",
                       "n": n, "steps": steps, "tol": 1e-28})
    out.update({"passes_per_step": [p["passes"] for p in per], "ms_per_step_each": [p["ms"] for p in per],
                "hp_ms_total": hp_ms, "quad_stril_rows_last": float(ev["stril"]),
                "quad_orth_rows_last": float(ev["orth"]), "steps": steps, "warmup": 0})
    out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                       "frac": achieved / INT8_PEAK_TOPS,
                       "traffic": pmc_traffic(f"dd_windows_n{n}_hbm_traffic.txt", "traffic_bytes_per_launch",
                                              OZAKI_SOURCES),
                       "traffic_unit": ("HBM bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, "
                                        "calibrated on a copy kernel)"),
                       "kernel": f"double-double product: the windowed INT8 product (oz_gemm_windows_kernel<0> "
                                 f"P = A Q and <2> That = Q^H P), {npairs} digit pairs x 8 n^3 ops per launch",
                       "avg_launch_ms": avg, "launches_per_step": cnt / steps}
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


def run_solvers(args) -> int:
    """The FP32 triangular-equation solve by the tile wavefront and by the recursive
    block algorithm (Algorithm 3, leaves of 64 and 256 rows) on the same data: T the
    upper triangular factor of a test matrix (gaps >= 0.05), E = 1e-6 CN(0,1) strictly
    lower, in complex64; milliseconds per solve (HIP events around each call, which
    ends with a synchronisation and the read of the status word)."""
    import torch

    import paper_2203_10879_amd as sr
    import synth

    sizes = [args.n] if args.n else [1024, 2048, 4096]
    torch.cuda.set_device(torch.device("cuda:0"))
    rows = []
    for n in sizes:
        g = synth.schur_test_matrix(n, seed=30 + n % 97)
        rng = np.random.default_rng(n)
        t = np.triu(g["T0"]).astype(np.complex64)
        e = (1e-6 * np.tril(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), -1)).astype(np.complex64)
        T, E = sr.colmajor(t), sr.colmajor(e)
        L = sr.colmajor_empty(n, n, torch.complex64)
        ws = sr.workspace(n)
        cases = {"wavefront": lambda: sr.sr_trisolve(T, E, L, ws)}
        for leaf in (64, 256):
            wr = torch.empty(int(sr.lib().sr_trisolve_rec_ws_bytes(n, leaf)), dtype=torch.uint8, device="cuda")
            cases[f"recursive_leaf{leaf}"] = (lambda wr=wr, leaf=leaf: sr.sr_trisolve_rec(T, E, L, leaf_rows=leaf,
                                                                                          ws=wr))
        row = {"n": n}
        for name, fn in cases.items():
            for _ in range(max(2, args.warmup)):
                assert fn() == 0
            ms = []
            for _ in range(args.steps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                rc = fn()
                e1.record()
                torch.cuda.synchronize()
                assert rc == 0
                ms.append(e0.elapsed_time(e1))
            row[name + "_ms"] = float(np.median(ms))
        print(f"# n={n}: " + ", ".join(f"{k} {v:.3f}" for k, v in row.items() if k != "n"), file=sys.stderr,
              flush=True)
        rows.append(row)
    best = rows[0]
    out = base_record(args, 1e3 / best["wavefront_ms"], "solves/s", best["wavefront_ms"], "c64",
                      {"workload": "FP32 triangular-equation solve, tile wavefront against the recursive block "
                                   "algorithm (Algorithm 3), T from a test matrix with gaps >= 0.05, "
                                   "E = 1e-6 CN(0,1)", "sizes": sizes})
    # The wavefront is a chain of dependent launches (one per tile diagonal): its rate
    # against the HBM peak (algorithmic bytes: the triangles of T and E read and of L
    # written, complex64) shows
    # how far the chain, not bandwidth, sets its time.
    n0 = best["n"]
    levels = -(-n0 // (16 if n0 <= 2048 else 32))
    alg = 12.0 * n0 * n0
    achieved = alg / (best["wavefront_ms"] * 1e-3) / 1e9
    out.update({"solves": rows})
    out["roofline"] = {"bound": "latency", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                       "frac": achieved / 8000.0,
                       "traffic": (pmc_traffic("trisolve_n1024_hbm_traffic.txt", "sweep_hbm_bytes_per_solve",
                                               SWEEP_SOURCES, "trisolve_source_sha256_16") if n0 == 1024 else None),
                       "traffic_unit": "HBM bytes per solve (rocprofv3 FETCH_SIZE and WRITE_SIZE)",
                       "kernel": f"triangular-equation sweep (trisolve_level_kernel<float>), {levels} dependent "
                                 f"launches at n = {n0}; algorithmic bytes 12 n^2 per solve",
                       "ms_per_solve": best["wavefront_ms"]}
    print(json.dumps(out), flush=True)
    return 0


REAL_SOURCES = ("real.hip", "real.hpp", "epilogue.hpp", "kernels.hpp", "common.hpp")


def run_real(args) -> int:
    """The real Schur variant: one real matrix with the spectrum structure of a real
    Gaussian matrix (about sqrt(2n/pi) real eigenvalues, the rest conjugate pairs in
    2 x 2 blocks, gaps >= 0.05, seed 3), started from the real Schur vectors of
    float32(A) (LAPACK sgees), FP64 tier to 1e-15."""
    import torch

    import oracle
    import paper_2203_10879_amd as sr
    import synth

    n = 2048 if args.n is None else args.n
    t0 = time.perf_counter()
    g = synth.real_schur_test_matrix(n, seed=3, gap=0.05)
    qh, blk = synth.lp_real_schur_start(g["A"])
    print(f"# inputs n={n} ready in {time.perf_counter() - t0:.1f} s ({int(blk.sum())} 2x2 blocks)",
          file=sys.stderr, flush=True)
    torch.cuda.set_device(torch.device("cuda:0"))
    A, Q0 = sr.colmajor(g["A"]), sr.colmajor(qh)
    Q, T = sr.colmajor_empty(n, n, torch.float64), sr.colmajor_empty(n, n, torch.float64)
    ws = sr.workspace_real(n)
    stream = torch.cuda.current_stream()

    def step(timing=False):
        Q.copy_(Q0)
        return sr.schur_refine_real(A, Q, T, blk, iters=8, tol=TOL, timing=timing, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    infos = []
    t1 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(step(timing=True))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    ok = all(i["status"] == "OK" for i in infos)
    steps = args.steps
    ms = sum(i["ms_hp_gemm"] - i["ms_hp_gemm_herm"] for i in infos)
    cnt = sum(i["hp_gemm_launches"] - i["hp_gemm_herm_launches"] for i in infos)
    herm = sum(i["hp_gemm_herm_launches"] for i in infos)
    avg = ms / max(1, cnt)
    achieved = 2.0 * n ** 3 / (avg * 1e-3) / 1e12
    last = infos[-1]
    out = base_record(args, steps / dt if ok else 0.0, "decomps/s", 1e3 * dt / steps, "f64",
                      {"workload": f"real Schur form, single real matrix n={n} (about sqrt(2n/pi) real "
                                   "eigenvalues, the rest conjugate pairs in 2x2 blocks, gaps >= 0.05, seed 3), "
                                   "FP32 sgees start, FP64 tier (FP64 MFMA products, FP32 block solve), "
                                   "tol 1e-15",
                       "n": n, "tol": TOL, "blocks_2x2": int(blk.sum()), "parallelism": "1 GPU"})
    out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / FP64_PEAK_TFLOPS,
                       "traffic": pmc_traffic(f"real_gemm_n{n}_hbm_traffic.txt", "traffic_bytes_per_launch",
                                              REAL_SOURCES),
                       "traffic_unit": ("HBM bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, "
                                        "calibrated on a copy kernel)"),
                       "kernel": "real FP64 GEMM (rgemm_kernel<double,...>), full products P, That, Q Delta: "
                                 "2n^3 flop per launch",
                       "avg_launch_ms": avg, "launches_per_step": cnt / steps,
                       "symmetric_products": {"launches_per_step": herm / steps,
                                              "avg_launch_ms": sum(i["ms_hp_gemm_herm"] for i in infos)
                                              / max(1, herm),
                                              "flop_per_launch": 1.0 * n * n * (n + 1)}}
    solves = sum(i["updates"] for i in infos)
    out.update({"passes": last["iters"], "hp_gemms": last["hp_gemms"], "resid_hist": last["resid_hist"],
                "ms_hp_gemm_per_step": sum(i["ms_hp_gemm"] for i in infos) / steps,
                "ms_solve_per_step": sum(i["ms_solve"] for i in infos) / steps,
                "ms_per_solve": sum(i["ms_solve"] for i in infos) / max(1, solves),
                "all_converged": ok})
    if args.rows > 0:
        # binary128 check on sampled rows: the block strictly lower entries of
        # Q_r^T A Q and the rows of Q_r^T Q - I
        step()
        torch.cuda.synchronize()
        q = sr.to_numpy(Q)
        rows = np.sort(np.random.default_rng(8).choice(n, args.rows, replace=False))
        qr = np.asfortranarray(q[:, rows]).astype(complex)
        rh, rl = oracle.gemm(qr, g["A"].astype(complex), opa=1).to_dd()
        mh, ml = oracle.gemm(np.asfortranarray(rh), q.astype(complex)).to_dd()
        m2h, m2l = oracle.gemm(np.asfortranarray(rl), q.astype(complex)).to_dd()
        m = (mh.real + m2h.real) + (ml.real + m2l.real)
        mask = np.tril(np.ones((n, n), dtype=bool), -1)[rows]
        for i in np.nonzero(blk)[0]:
            mask[rows == i + 1, i] = False
        stril = float(np.sqrt(np.sum(m[mask] ** 2) * n / len(rows)) / np.linalg.norm(g["A"]))
        oh, ol = oracle.gemm(qr, q.astype(complex), opa=1).to_dd()
        o = oh.real.copy()
        o[np.arange(len(rows)), rows] -= 1.0
        o += ol.real
        out.update({"quad_stril_rows": stril, "quad_orth_rows": float(np.sqrt(np.sum(o ** 2) * n / len(rows))),
                    "quad_rows": int(args.rows)})
        out["all_converged"] = ok and stril <= TOL
    print(json.dumps(out), flush=True)
    return 0 if out["all_converged"] else 1


TD_TOL = 1e-42


def run_td(args) -> int:
    """The triple-double tier: one complex matrix (gaps >= 0.05, seed 6) from its
    complex128 Schur basis (LAPACK zgees) to 1e-42, every hp value three complex128
    terms, hp products from 20 INT8 digits per operand, FP64 solve and lp products."""
    import torch

    import paper_2203_10879_amd as sr
    import synth
    from oracle import exact

    n = 1024 if args.n is None else args.n
    t0 = time.perf_counter()
    g = synth.schur_test_matrix(n, seed=6, gap=0.05)
    qh = synth.hp_schur_start(g["A"])
    print(f"# inputs n={n} ready in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.set_device(torch.device("cuda:0"))
    z = np.zeros_like(g["A"])
    As = [sr.colmajor(g["A"]), sr.colmajor(z), sr.colmajor(z)]
    starts = [sr.colmajor(qh), sr.colmajor(z), sr.colmajor(z)]
    Qs = [sr.colmajor_empty(n, n) for _ in range(3)]
    Ts = [sr.colmajor_empty(n, n) for _ in range(3)]
    ws = torch.empty(int(sr.lib().sr_workspace_bytes_td(n, None)), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step(timing=False):
        for q, q0 in zip(Qs, starts):
            q.copy_(q0)
        return sr.schur_refine_td(As, Qs, Ts, iters=8, tol=TD_TOL, timing=timing, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    infos = []
    t1 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(step(timing=True))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    ok = all(i["status"] == "OK" for i in infos)
    steps = args.steps
    # the product launches P = A Q and That alone (HIP events on the library's stream)
    ms = sum(i["ms_oz_full"] for i in infos)
    cnt = sum(i["oz_full_launches"] for i in infos)
    avg = ms / max(1, cnt)
    pairs = infos[-1]["oz_full_pairs"]
    achieved = pairs * 8.0 * n ** 3 / (avg * 1e-3) / 1e12
    last = infos[-1]
    out = base_record(args, steps / dt if ok else 0.0, "decomps/s", 1e3 * dt / steps, "td(int8)",
                      {"workload": f"triple-double tier, single matrix n={n}, eigenvalue gaps >= 0.05 (seed 6), "
                                   "complex128 zgees start, tol 1e-42 (three complex128 terms per hp value, "
                                   "20 INT8 digits per operand, FP64 solve)",
                       "n": n, "tol": TD_TOL, "parallelism": "1 GPU"})
    out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                       "frac": achieved / INT8_PEAK_TOPS,
                       "traffic": pmc_traffic(f"td_windows_n{n}_hbm_traffic.txt", "traffic_bytes_per_launch",
                                              OZAKI_SOURCES),
                       "traffic_unit": ("HBM bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, "
                                        "calibrated on a copy kernel)"),
                       "kernel": f"triple-double product: the windowed INT8 product with three-term outputs "
                                 f"(oz_gemm_windows_kernel<0> P = A Q and <2> That = Q^H P), {pairs} digit pairs "
                                 f"x 8 n^3 ops per launch",
                       "avg_launch_ms": avg, "launches_per_step": cnt / steps,
                       "with_splits_ms": sum(i["ms_hp_gemm"] - i["ms_hp_gemm_herm"] for i in infos)
                       / max(1, sum(i["hp_gemm_launches"] - i["hp_gemm_herm_launches"] for i in infos))}
    out.update({"passes": last["iters"], "hp_gemms": last["hp_gemms"], "resid_hist": last["resid_hist"],
                "ms_hp_gemm_per_step": sum(i["ms_hp_gemm"] for i in infos) / steps,
                "ms_solve_per_step": sum(i["ms_solve"] for i in infos) / steps, "all_converged": ok})
    r = min(args.rows, 2)
    if r > 0:
        # exact check (Python integers) on sampled rows of the last refinement
        step()
        torch.cuda.synchronize()
        rows = np.sort(np.random.default_rng(10).choice(n, r, replace=False))
        t2 = time.perf_counter()
        ev = exact.residual_rows([g["A"]], [sr.to_numpy(q) for q in Qs], rows)
        print(f"# exact rows checked in {time.perf_counter() - t2:.1f} s", file=sys.stderr, flush=True)
        out.update({"exact_stril_rows": ev["stril"], "exact_orth_rows": ev["orth"], "exact_rows": r})
        out["all_converged"] = ok and ev["stril"] <= TD_TOL and ev["orth"] <= TD_TOL
    print(json.dumps(out), flush=True)
    return 0 if out["all_converged"] else 1


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="matrix size (default: the workload's)")
    ap.add_argument("--workload", default="default",
                    choices=["default", "single", "precision", "batched", "dd_continuation", "real", "solvers",
                             "td"])
    ap.add_argument("--count", type=int, default=2000, help="batched: number of matrices")
    ap.add_argument("--cont-steps", type=int, default=64, help="dd_continuation: steps")
    ap.add_argument("--rows", type=int, default=32, help="rows of the binary128 check")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="default: leave out the n = 1024 key")
    ap.add_argument("--forms", default="", help="default: comma-separated forms to run (default: all four)")
    ap.add_argument("--no-compensated", action="store_true")
    ap.add_argument("--lp-digits", type=int, default=4,
                    help="split forms: INT8 digits of the lp products (0: FP32 MFMA)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the refinement of one matrix is not sharded across GPUs)",
              file=sys.stderr)
        return 2
    return {"default": run_default, "single": run_single, "precision": run_precision, "batched": run_batched,
            "dd_continuation": run_dd_continuation, "real": run_real, "solvers": run_solvers,
            "td": run_td}[args.workload](args)


if __name__ == "__main__":
    sys.exit(main())
