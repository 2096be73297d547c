#!/usr/bin/env python3
"""Time-to-solution of scale-and-fold purification vs the trace-correcting scheme on MI355X.

One step = one complete purification D = theta(mu I - F) of the two-orbital cubic
tight-binding lattice with 16x16x8 sites (n = 4096, half filling) in FP64, from f_0 through
the product that certifies ||X^2 - X||_F <= 1e-8, with F already resident in HBM.  The timed
scheme is the varying-mu scale-and-fold scheme (Algorithm 2); the unscaled trace-correcting
scheme (x^2 / 2x - x^2 chosen by the trace) is timed the same way beside it.

Prints one JSON line.  Extra keys:
  roofline      dominant kernel (the FP64 MFMA X.X product) against the FP64 MFMA peak;
                algorithmic flops n^2 (n + 1) per product (the symmetric product needs only
                the upper triangle), average product-kernel duration from HIP events recorded
                on the library's stream over the timed solves;
  cpu_baseline  the FP64 CPU oracle (numpy) on the same workload, one solve, host cores;
  workloads     compact objects for the other four workloads, each with its own value,
                roofline and cpu_baseline: n = 256 with a 0.05 gap (latency), n = 8192 with a
                1e-3 gap (FP64 against FP32/BF16 products with FP64 refinement), the
                block-sparse lattice n = 65536, and the 512-request serving trace.  Their own
                --workload lines give the full detail.
"""
import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time-to-solution ms at ‖X²−X‖≤1e-8, SnF vs SP2; "
          "X·X TFLOP/s & GB/s")
PEAK_FP64_TFLOPS = 78.6
TOL = 1e-8
LATTICE = (16, 16, 8)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "xx_f64_lattice_n4096_traffic.json")


def _code_only(text: str) -> str:
    """Source text without comments and with whitespace collapsed: the hash follows the code
    the counters measured, not its comments."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(files=("kernels_dense.hip", "snf_internal.h", "schedule_math.h")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1101_0265_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


BSR_SOURCES = ("bsr.hip", "kernels_dense.hip", "snf_internal.h", "schedule_math.h")
BSR_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bsr_lattice_n65536_traffic.json")


def load_bsr_traffic():
    """Counter-measured bytes and time of the block-sparse product kernel for the solves of
    the block-sparse workload, or None if taken on other sources."""
    try:
        with open(BSR_TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash(BSR_SOURCES):
        return None
    return t


def load_traffic(n_products_per_launch: int = 1):
    """HBM bytes per product launch from the committed rocprofv3 counter summary, or None
    if it was taken on a different version of the kernels."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(h, kw):
    import numpy as np
    from oracle import dense
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 1) for i in threadpool_info()
                       if i.get("user_api") == "blas"), default=os.cpu_count())
    except Exception:  # noqa: BLE001
        threads = os.cpu_count()
    t0 = time.perf_counter()
    r = dense.purify(h.F, "snf_varmu", **kw)
    dt = time.perf_counter() - t0
    out = dict(value=round(dt * 1e3, 1), unit="ms", cores=int(threads), kind="oracle",
               sample=("one full solve of the same workload (n=4096 lattice, SnF varying-mu, "
                       f"FP64 numpy, {r['products']} method products; the oracle also forms "
                       "X^2 separately for its check)"))
    # the same oracle on one core: its first iteration (a check and a step, 3 dense
    # products), scaled to the solve's 2 * iterations + 1 products
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1, user_api="blas"):
            t0 = time.perf_counter()
            dense.purify(h.F, "snf_varmu", **dict(kw, tol=1e-300, max_iter=1))
            dt1 = time.perf_counter() - t0
        its = r["iterations"]
        out["single_core"] = dict(
            value=round(dt1 * 1e3 * (2 * its + 1) / 3, 1), unit="ms", cores=1,
            sample=f"first iteration on one core ({dt1:.1f} s for 3 dense products), scaled to "
                   f"the solve's {2 * its + 1}")
    except Exception as exc:  # noqa: BLE001
        out["single_core"] = dict(value=None, note=f"not measured: {exc}")
    return out


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max((i.get("num_threads", 1) for i in threadpool_info()
                    if i.get("user_api") == "blas"), default=os.cpu_count())
    except Exception:  # noqa: BLE001
        return os.cpu_count()


def _base_line(metric, value, unit, args, higher, dtype, config):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": None, "higher_is_better": higher,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": config}


def run_small(args):
    """n = 256, gap 0.05 about mu = 0, tol 1e-10: latency of each scheme (FP64)."""
    import torch
    from paper_1101_0265_amd import hamiltonians as H
    from paper_1101_0265_amd import snf
    h = H.small_gap_256()
    F = torch.tensor(h.F, device="cuda:0")
    D = torch.empty_like(F)
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
              lumo=h.lumo, mu=h.mu, xi=h.xi, tol=1e-10, max_iter=100)
    out = {}
    # a solve takes well under a millisecond, so single outliers (a clock ramp, a host
    # hiccup) move a mean of a few solves: each solve is timed on its own (the call returns
    # after its result is read back) and the median of at least 20 is reported
    reps = max(args.steps, 20)
    for scheme in ("snf_varmu", "snf_fixmu", "sp2", "tc2", "mcweeny", "snf_fixmu3",
                   "snf_fixmu5", "pmm3", "pmm5"):
        for _ in range(max(args.warmup, 3)):
            snf.purify_dense(F, scheme, out=D, want_log=False, **kw)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            _, r = snf.purify_dense(F, scheme, out=D, want_log=False, **kw)
            times.append((time.perf_counter() - t0) * 1e3)
        torch.cuda.synchronize()
        times.sort()
        out[scheme] = dict(ms=round(times[len(times) // 2], 4),
                           mean_ms=round(sum(times) / len(times), 4), solves=reps,
                           products=r["products"], status=r["status"],
                           device_ms=round(r["device_ms"], 4))
    line = _base_line("time-to-solution ms at ‖X²−X‖≤1e-10, SnF vs SP2 (n=256)",
                      out["snf_varmu"]["ms"], "ms", args, False, "f64",
                      {"workload": "dense FP64 n=256, spectrum [-1,-0.025] u [0.025,1], Haar Q "
                                   "(seed 1101), N_occ=128, tol 1e-10"})
    line["ms_per_step"] = out["snf_varmu"]["ms"]
    line["schemes"] = out
    line["speedup_vs_sp2"] = round(out["sp2"]["ms"] / out["snf_varmu"]["ms"], 3)
    # the product kernel of this order (32x32 tiles, k split inside the workgroup), timed with
    # HIP events around every product launch of one solve
    _, rt = snf.purify_dense(F, "snf_varmu", out=D, want_log=False,
                             flags=snf.FLAG_TIME_PRODUCTS, **kw)
    n = h.n
    achieved = rt["products"] * float(n) * n * (n + 1) / rt["product_ms"] / 1e9
    line["roofline"] = dict(bound="mfma", achieved=round(achieved, 3), peak=78.6,
                            unit="TFLOP/s", frac=round(achieved / 78.6, 5), traffic=None,
                            kernel="product_f64_small_kernel (32x32 tiles, n=256)",
                            avg_launch_us=round(rt["product_ms"] * 1e3 / rt["products"], 2),
                            note="n^2 (n+1) flops per product over the HIP-event time of its "
                                 "launch; at this order a launch is latency-bound (36 "
                                 "workgroups of 1.1 MFLOP each)")
    from oracle import dense
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        dense.purify(h.F, "snf_varmu", **kw)
    cpu_ms = (time.perf_counter() - t0) * 1e3 / reps
    line["cpu_baseline"] = dict(value=round(cpu_ms, 3), unit="ms", cores=int(_blas_threads()),
                                kind="oracle", sample=f"{reps} solves of the same n=256 input")
    return line


def run_precision(args):
    """n = 8192, spectrum in [-1, 1] with a 1e-3 gap at mu = 0.1 (N_occ = 4506), Haar Q:
    FP64 against FP32 / BF16 products with FP64 refinement, each solve's distance to the
    exact projector Q_occ Q_occ^T."""
    import numpy as np
    import torch
    from paper_1101_0265_amd import hamiltonians as H
    from paper_1101_0265_amd import snf
    n, n_occ = 8192, 4506
    lam = H.two_interval_spectrum(n_occ, n - n_occ, -1.0, 0.0995, 0.1005, 1.0,
                                  np.random.default_rng(4))
    F, Q = H.rotated_spectrum_torch(lam, seed=4)
    qo = Q[:, :n_occ].contiguous()
    D_exact = qo @ qo.T
    del Q, qo
    D = torch.empty_like(F)
    kw = dict(lambda_min=-1.0, lambda_max=1.0, n_occ=n_occ, homo=0.0995, lumo=0.1005, mu=0.1,
              xi=1e-3, tol=1e-8, max_iter=200)
    runs = [("snf_varmu", "fp64", 0.0), ("sp2", "fp64", 0.0), ("snf_fixmu", "fp64", 0.0),
            ("snf_fixmu3", "fp64", 0.0), ("snf_fixmu5", "fp64", 0.0), ("mcweeny", "fp64", 0.0),
            ("snf_varmu", "fp32_ref64", 0.0), ("snf_varmu", "fp32_ref64", 0.5),
            ("snf_varmu", "fp32_ref64", 0.9), ("snf_varmu", "bf16_ref64", 0.5),
            ("snf_varmu", "bf16_ref64", 0.9), ("snf_varmu", "fp32", 0.0)]
    if getattr(args, "compact", False):
        runs = [("snf_varmu", "fp64", 0.0), ("sp2", "fp64", 0.0), ("snf_fixmu", "fp64", 0.0),
                ("snf_varmu", "fp32_ref64", 0.0), ("snf_varmu", "fp32_ref64", 0.5),
                ("snf_varmu", "bf16_ref64", 0.5)]
    # the FP32 and BF16 modes again with the subspace correction (one Newton step that
    # re-references F, then FP64 refinement)
    runs = [(sc, pr, g, 0) for sc, pr, g in runs] + [
        ("snf_varmu", "fp32_ref64", 0.0, snf.FLAG_SUBSPACE_NEWTON),
        ("snf_varmu", "fp32_ref64", 0.5, snf.FLAG_SUBSPACE_NEWTON),
        ("snf_varmu", "bf16_ref64", 0.5, snf.FLAG_SUBSPACE_NEWTON)]
    out = {}
    for scheme, prec, gsw, fl in runs:
        snf.purify_dense(F, scheme, prec, out=D, want_log=False, gap_switch=gsw, flags=fl, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = max(1, args.steps)
        for _ in range(steps):
            _, r = snf.purify_dense(F, scheme, prec, out=D, want_log=False, gap_switch=gsw,
                                    flags=fl, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        err = float(torch.linalg.norm(D - D_exact))
        comm = float(torch.linalg.norm(F @ D - D @ F))
        out[f"{scheme}/{prec}/gsw{gsw}" + ("/newton" if fl else "")] = dict(
            ms=round(ms, 2), status=r["status"], products=r["products"],
            products_fp64=r["products_fp64"], products_lowp=r["products_lowp"],
            products_newton=r["products_newton"], idem_err=r["idem_err"],
            trace_err=r["trace_err"], dist_to_exact_D=err, commutator=comm)
    flops_one = float(n) * n * (n + 1)
    # FP64 product kernel: every product of the FP64 scale-and-fold solve timed
    _, r64 = snf.purify_dense(F, "snf_varmu", "fp64", out=D, want_log=False,
                              flags=snf.FLAG_TIME_PRODUCTS, **kw)
    f64_tflops = r64["products"] * flops_one / r64["product_ms"] / 1e9
    # FP32 product kernel alone: the FP32-only mode from the start, every product timed
    _, rf = snf.purify_dense(F, "snf_varmu", "fp32", out=D, want_log=False, gap_switch=0.0,
                             flags=snf.FLAG_TIME_PRODUCTS, **kw)
    f32_tflops = rf["products"] * flops_one / rf["product_ms"] / 1e9
    # BF16 product kernel: one step X.X on the FP64 solve's D (the stand-alone product)
    bf_ms = []
    for _ in range(4):
        _, _, kms = snf.step_dense(D, D, 1.0, 0.0, 0.0, "bf16_ref64")
        bf_ms.append(kms)
    bf_ms = sorted(bf_ms)[len(bf_ms) // 2]
    bf16_tflops = flops_one / bf_ms / 1e9
    base = out["snf_varmu/fp64/gsw0.0"]
    line = _base_line("time-to-solution ms at ‖X²−X‖≤1e-8 by precision mode (n=8192)",
                      base["ms"], "ms", args, False, "f64",
                      {"workload": "dense n=8192, Haar Q, spectrum uniform in [-1,1] with a 1e-3 "
                                   "gap at mu=0.1, N_occ=4506, tol 1e-8; FP64 vs FP32/BF16 "
                                   "products + FP64 refinement"})
    line["ms_per_step"] = base["ms"]
    line["runs"] = out
    line["speedup_vs_sp2"] = round(out["sp2/fp64/gsw0.0"]["ms"] / base["ms"], 3)
    line["roofline"] = dict(bound="mfma", achieved=round(f64_tflops, 2), peak=78.6,
                            unit="TFLOP/s", frac=round(f64_tflops / 78.6, 4), traffic=None,
                            kernel="product_f64_kernel (f64 MFMA, 128x128 tiles, n=8192)",
                            avg_launch_ms=round(r64["product_ms"] / r64["products"], 3),
                            note="n^2 (n+1) flops per product over the HIP-event time of the "
                                 "product launches of the FP64 scale-and-fold solve")
    line["roofline_fp32"] = dict(bound="mfma", achieved=round(f32_tflops, 2), peak=157.3,
                                 unit="TFLOP/s", frac=round(f32_tflops / 157.3, 4),
                                 kernel="product_f32_kernel (f32 MFMA, n=8192)",
                                 avg_launch_ms=round(rf["product_ms"] / rf["products"], 3),
                                 note="every product of an FP32-only solve timed (the FP32 "
                                      "products of the refined modes run the same kernel)")
    line["roofline_bf16"] = dict(bound="mfma", achieved=round(bf16_tflops, 1), peak=2500.0,
                                 unit="TFLOP/s", frac=round(bf16_tflops / 2500.0, 4),
                                 kernel="product_bf16_kernel (bf16 MFMA, f32 accumulation, "
                                        "n=8192)",
                                 avg_launch_ms=round(bf_ms, 3),
                                 note="one stand-alone product X.X (snf_step_dense), median "
                                      "of 4 HIP-event kernel times")
    line["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        # the oracle on the same F for its first two iterations, scaled per iteration to the
        # solve's iteration count (its per-iteration cost is the same at every iteration)
        from oracle import dense
        Fh = F.cpu().numpy()
        okw = {k: v for k, v in kw.items() if k in ("lambda_min", "lambda_max", "n_occ", "homo",
                                                     "lumo", "mu", "xi")}
        t0 = time.perf_counter()
        dense.purify(Fh, "snf_varmu", tol=1e-300, max_iter=2, **okw)
        dt = time.perf_counter() - t0
        its = base["products"] - 1
        line["cpu_baseline"] = dict(
            value=round(dt * 1e3 * (2 * its + 1) / 5, 1), unit="ms", cores=int(_blas_threads()),
            kind="oracle",
            sample=f"the first 2 iterations of the FP64 oracle on the same n=8192 F (5 dense "
                   f"products: 3 checks, 2 steps; {dt:.1f} s), scaled to the solve's "
                   f"{2 * its + 1} ({its} iterations of check + step, one certifying check)")
    return line


def run_fixmu(args):
    """n = 4096, spectrum in [-1, 1] with a 0.01 gap centred at mu = -0.5 (a quarter of the
    way up; N_occ = 1024), Haar Q: the fixed-mu schemes -- Algorithm 1 (P_{1,1}), P_{m,m},
    and P_{i,j} (i != j) scaled about its fixed point x* -- and their alpha = 1 forms."""
    import numpy as np
    import torch
    from paper_1101_0265_amd import hamiltonians as H
    from paper_1101_0265_amd import snf
    n, mu, gap = 4096, -0.5, 0.01
    n_occ = int(round(n * (mu + 1.0) / 2.0))
    lam = H.two_interval_spectrum(n_occ, n - n_occ, -1.0, mu - gap / 2, mu + gap / 2, 1.0,
                                  np.random.default_rng(11))
    F, Q = H.rotated_spectrum_torch(lam, seed=11)
    qo = Q[:, :n_occ].contiguous()
    D_exact = qo @ qo.T
    del Q, qo
    D = torch.empty_like(F)
    kw = dict(lambda_min=-1.0, lambda_max=1.0, n_occ=n_occ, mu=mu, xi=gap, tol=1e-8,
              max_iter=120, flags=snf.FLAG_TIME_PRODUCTS)
    runs = [("snf_fixmu", None), ("mcweeny", None), ("snf_fixmu3", None), ("snf_fixmu5", None),
            ("snf_pij", (3, 1)), ("snf_pij", (1, 3)), ("snf_pij", (5, 1)), ("snf_pij", (1, 5)),
            ("snf_pij", (5, 3)), ("snf_pij", (3, 5)), ("pij", (3, 1)), ("pij", (1, 3))]
    flops_one = float(n) * n * (n + 1)
    out = {}
    for scheme, pij in runs:
        name = scheme + ("" if pij is None else f"{pij[0]}{pij[1]}")
        snf.purify_dense(F, scheme, out=D, want_log=False, poly_ij=pij, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = max(1, args.steps)
        for _ in range(steps):
            _, r = snf.purify_dense(F, scheme, out=D, want_log=False, poly_ij=pij, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        out[name] = dict(ms=round(ms, 2), status=r["status"], products=r["products"],
                         iterations=r["iterations"], idem_err=r["idem_err"],
                         trace_err=r["trace_err"],
                         dist_to_exact_D=float(torch.linalg.norm(D - D_exact)),
                         product_ms=round(r["product_ms"], 2),
                         product_tflops=round(r["products"] * flops_one / r["product_ms"] / 1e9,
                                              2))
    base = out["snf_pij31"]
    line = _base_line("time-to-solution ms at ‖X²−X‖≤1e-8, fixed-mu schemes, mu off-centre "
                      "(n=4096)", base["ms"], "ms", args, False, "f64",
                      {"workload": "dense FP64 n=4096, Haar Q (seed 11), spectrum uniform in "
                                   "[-1,1] with a 0.01 gap centred at mu=-0.5, N_occ=1024, "
                                   "tol 1e-8"})
    line["ms_per_step"] = base["ms"]
    line["runs"] = out
    line["speedup_vs_mcweeny"] = round(out["mcweeny"]["ms"] / base["ms"], 3)
    achieved = base["product_tflops"]
    line["roofline"] = dict(bound="mfma", achieved=achieved, peak=78.6, unit="TFLOP/s",
                            frac=round(achieved / 78.6, 4), traffic=None,
                            kernel="product_f64_kernel and product_f64_dual_kernel (P_{3,1})",
                            note="n^2 (n+1) flops per product over the summed HIP-event time "
                                 "of the product launches of one solve")
    line["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        # one iteration of the oracle on the same F (the check X^2 and the four Horner
        # products of P_{3,1} in X_s), scaled to the solve's iterations
        from oracle import dense
        Fh = F.cpu().numpy()
        okw = dict(lambda_min=-1.0, lambda_max=1.0, n_occ=n_occ, mu=mu, xi=gap)
        t0 = time.perf_counter()
        dense.purify(Fh, "snf_pij", tol=1e-300, max_iter=1, poly_ij=(3, 1), **okw)
        dt = time.perf_counter() - t0
        its = base["iterations"]
        line["cpu_baseline"] = dict(
            value=round(dt * 1e3 * (5 * its + 1) / 6, 1), unit="ms", cores=int(_blas_threads()),
            kind="oracle",
            sample=f"one iteration of the FP64 oracle on the same n=4096 F (6 dense products: "
                   f"2 checks, 4 Horner steps; {dt:.1f} s), scaled to the solve's "
                   f"{5 * its + 1} ({its} iterations of check + 4 steps, one certifying check)")
    return line


def run_bounds(args):
    """n = 4096 lattice: bounds estimated on the device (Lanczos, 40 steps) instead of given.
    The trace scheme with estimated extremal bounds, gap bounds from its D, then scale-and-fold
    with them; against the solve with exact bounds."""
    import numpy as np
    import torch
    from paper_1101_0265_amd import hamiltonians as H
    from paper_1101_0265_amd import snf
    h = H.lattice_hamiltonian((16, 16, 8), seed=2)
    F = torch.tensor(h.F, device="cuda:0")
    D1, D2 = torch.empty_like(F), torch.empty_like(F)
    steps = 40
    exact_kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ,
                    homo=h.homo, lumo=h.lumo, tol=1e-8, max_iter=100)

    def pipeline():
        lo, hi, glo, ghi = snf.spectral_bounds(F, steps)
        _, r1 = snf.purify_dense(F, "sp2", out=D1, want_log=False, lambda_min=lo,
                                 lambda_max=hi, n_occ=h.n_occ, tol=1e-8, max_iter=100)
        homo, lumo = snf.gap_bounds(F, D1, lo, hi, steps)
        _, r2 = snf.purify_dense(F, "snf_varmu", out=D2, want_log=False, lambda_min=lo,
                                 lambda_max=hi, homo=homo, lumo=lumo, n_occ=h.n_occ,
                                 tol=1e-8, max_iter=100)
        return (lo, hi, glo, ghi, homo, lumo), r1, r2

    for _ in range(max(1, args.warmup)):
        pipeline()
    torch.cuda.synchronize()
    t = {}
    t0 = time.perf_counter()
    snf.spectral_bounds(F, steps)
    torch.cuda.synchronize()
    t["spectral_bounds_ms"] = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    snf.gap_bounds(F, D1, h.lambda_min, h.lambda_max, steps)
    torch.cuda.synchronize()
    t["gap_bounds_ms"] = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    b, r1, r2 = pipeline()
    torch.cuda.synchronize()
    t["pipeline_ms"] = (time.perf_counter() - t0) * 1e3
    b_est = (b[0], b[1], b[4], b[5])
    t0 = time.perf_counter()
    _, rx = snf.purify_dense(F, "snf_varmu", out=D2, want_log=False, **exact_kw)
    torch.cuda.synchronize()
    t["snf_exact_bounds_ms"] = (time.perf_counter() - t0) * 1e3
    # the pipeline's dominant kernel, the FP64 product: the SnF solve with estimated bounds,
    # every product timed
    _, rt = snf.purify_dense(F, "snf_varmu", out=D2, want_log=False,
                             flags=snf.FLAG_TIME_PRODUCTS, lambda_min=b_est[0],
                             lambda_max=b_est[1], homo=b_est[2], lumo=b_est[3],
                             n_occ=h.n_occ, tol=1e-8, max_iter=100)
    w = np.linalg.eigvalsh(h.F)
    line = _base_line("time ms: bounds estimated on the device, then SP2 and SnF (n=4096)",
                      round(t["pipeline_ms"], 2), "ms", args, False, "f64",
                      {"workload": "dense FP64 two-orbital lattice 16x16x8 sites, n=4096; "
                                   f"Lanczos {steps} steps for extremal and gap bounds"})
    line["ms_per_step"] = line["value"]
    line["timings_ms"] = {k: round(v, 2) for k, v in t.items()}
    line["bounds"] = dict(lambda_min=b[0], lambda_max=b[1], gershgorin=[b[2], b[3]],
                          homo=b[4], lumo=b[5], exact=[float(w[0]), float(w[-1]), h.homo,
                                                        h.lumo])
    line["products"] = dict(sp2_estimated=r1["products"], snf_estimated=r2["products"],
                            snf_exact=rx["products"])
    nn = h.n
    achieved = rt["products"] * float(nn) * nn * (nn + 1) / rt["product_ms"] / 1e9
    line["roofline"] = dict(bound="mfma", achieved=round(achieved, 2), peak=78.6,
                            unit="TFLOP/s", frac=round(achieved / 78.6, 4), traffic=None,
                            kernel="product_f64_kernel (the pipeline's dominant kernel)",
                            note="n^2 (n+1) flops per product over the HIP-event time of the "
                                 "products of the SnF solve with estimated bounds; the "
                                 "Lanczos matrix-vector product is HBM-bound (68.2 MB per "
                                 "launch)")
    line["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        from oracle import bounds as obounds, dense
        v0 = np.random.default_rng(0).standard_normal(h.n)
        t0 = time.perf_counter()
        lo, hi = obounds.spectral_bounds(h.F, v0, steps)
        o1 = dense.purify(h.F, "sp2", lambda_min=lo, lambda_max=hi, n_occ=h.n_occ, tol=1e-8,
                          max_iter=100)
        homo, lumo = obounds.gap_bounds(h.F, o1["D"], lo, hi, v0, steps)
        dense.purify(h.F, "snf_varmu", lambda_min=lo, lambda_max=hi, homo=homo, lumo=lumo,
                     n_occ=h.n_occ, tol=1e-8, max_iter=100)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = dict(value=round(dt * 1e3, 1), unit="ms",
                                    cores=int(_blas_threads()), kind="oracle",
                                    sample="the whole pipeline once on the same input "
                                           "(numpy Lanczos, FP64 oracle solves)")
    return line


def _bsr_mm(rp, ci, va, Z):
    """Y = M Z for a BSR matrix M (32x32 blocks, device tensors) and a dense (n, p) float64
    block of vectors, by batched block products (measurement helper)."""
    import torch
    nb = rp.numel() - 1
    p = Z.shape[1]
    rows = torch.repeat_interleave(torch.arange(nb, device=Z.device), rp[1:] - rp[:-1])
    Zb = Z.reshape(nb, 32, p)
    out = torch.zeros(nb, 32, p, dtype=torch.float64, device=Z.device)
    step = 65536
    for c0 in range(0, ci.numel(), step):
        c1 = min(c0 + step, ci.numel())
        G = Zb[ci[c0:c1].long()].contiguous()
        V = va[c0:c1].double().contiguous()
        out.index_add_(0, rows[c0:c1], torch.bmm(V, G))
    return out.reshape(nb * 32, p)


def _bsr_commutator(Fm, Dm, n, probes=4, seed=0):
    """Hutchinson estimate of ||F D - D F||_F: E ||[F, D] z||^2 over Gaussian z."""
    import torch
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    Z = torch.randn(n, probes, generator=g, device="cuda:0", dtype=torch.float64)
    C = _bsr_mm(*Fm, _bsr_mm(*Dm, Z)) - _bsr_mm(*Dm, _bsr_mm(*Fm, Z))
    return float(torch.sqrt((C * C).sum() / probes))


def run_bsr(args):
    """Block-sparse lattice 32x32x32 sites (n = 65536, 32x32 FP32 blocks, tau = 1e-6):
    time to the truncation floor, SnF varying-mu vs the trace scheme."""
    import numpy as np
    import torch
    from paper_1101_0265_amd import hamiltonians as H
    from paper_1101_0265_amd import snf
    L = (32, 32, 32)
    m, h = H.lattice_bsr(L, seed=3)
    rp = torch.tensor(m.row_ptr, device="cuda:0")
    ci = torch.tensor(m.col_idx, device="cuda:0")
    va = torch.tensor(m.val, device="cuda:0")
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
              lumo=h.lumo, tol=1e-9, max_iter=80, flags=snf.FLAG_TIME_PRODUCTS)
    if args.bsr_sweep:
        D, _ = snf.purify_bsr(rp, ci, va, m.n, "snf_varmu", trunc_tau=1e-5, want_log=False, **kw)
        del D
        for scheme, tau in (("sp2", 1e-6), ("sp2", 3e-7), ("snf_varmu", 1e-6),
                            ("snf_varmu", 2e-6), ("snf_varmu", 5e-6), ("snf_varmu", 1e-5),
                            ("tc2", 1e-6)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            D, r = snf.purify_bsr(rp, ci, va, m.n, scheme, trunc_tau=tau, **kw)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            peak = max(x["phase"] for x in r["log"]) / m.nb
            print(json.dumps(dict(scheme=scheme, tau=tau, ms=round(ms, 1),
                                  products=r["products"], status=r["status"],
                                  e=r["idem_err"], trace_err=r["trace_err"],
                                  blocks_per_row=round(r["blocks"] / m.nb, 1),
                                  peak_blocks_per_row=round(peak, 1))), flush=True)
            del D
    if args.bsr_fixmu:
        # Algorithm 1 (two products per iteration, truncation after the second) beside
        # Algorithm 2 and the trace scheme, tau = 1e-6, unscreened and norm-screened at 1e-8;
        # accuracy from ||[F, D]||_F
        kw1 = dict(kw, mu=h.mu, xi=h.xi)
        for scheme, sigma in [(sc, sg) for sg in (0.0, 1e-8)
                              for sc in ("snf_fixmu", "snf_varmu", "sp2")]:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            D, r = snf.purify_bsr(rp, ci, va, m.n, scheme, trunc_tau=1e-6,
                                  **dict(kw1, screen_tau=sigma))
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            comm = _bsr_commutator((rp, ci, va), D, m.n)
            peak = max(x["phase"] for x in r["log"]) / m.nb
            print(json.dumps(dict(scheme=scheme, tau=1e-6, screen_tau=sigma, ms=round(ms, 1),
                                  products=r["products"], iterations=r["iterations"],
                                  status=r["status"], e=r["idem_err"],
                                  trace_err=r["trace_err"], commutator=comm,
                                  product_ms=round(r["product_ms"], 1),
                                  blocks_per_row=round(r["blocks"] / m.nb, 1),
                                  peak_blocks_per_row=round(peak, 1))), flush=True)
            del D
    if args.bsr_ec:
        # fixed threshold against error-controlled truncation at several budgets; accuracy
        # from ||[F, D]||_F (no exact D at this size)
        D, _ = snf.purify_bsr(rp, ci, va, m.n, "tc2", trunc_tau=1e-2, want_log=False,
                              **dict(kw, flags=kw["flags"] | snf.FLAG_TRUNC_ERROR_CONTROL))
        del D
        runs = [(sc, "tau", 1e-6) for sc in ("tc2", "snf_varmu", "snf_fixmu")]
        runs += [(sc, "eps", e) for sc in ("tc2", "snf_varmu", "snf_fixmu")
                 for e in (1e-1, 3e-2, 1e-2, 3e-3)]
        for scheme, kind, val in runs:
            fl = kw["flags"] | (snf.FLAG_TRUNC_ERROR_CONTROL if kind == "eps" else 0)
            skw = dict(kw, flags=fl)
            if scheme == "snf_fixmu":                  # Algorithm 1: mu mid-gap, xi the gap
                skw.update(mu=h.mu, xi=h.xi)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            D, r = snf.purify_bsr(rp, ci, va, m.n, scheme, trunc_tau=val, **skw)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            comm = _bsr_commutator((rp, ci, va), D, m.n)
            peak = max(x["phase"] for x in r["log"]) / m.nb
            print(json.dumps(dict(scheme=scheme, rule=kind, value=val, ms=round(ms, 1),
                                  products=r["products"], status=r["status"],
                                  e=r["idem_err"], trace_err=r["trace_err"], commutator=comm,
                                  blocks_per_row=round(r["blocks"] / m.nb, 1),
                                  peak_blocks_per_row=round(peak, 1))), flush=True)
            del D
    if args.bsr_screen:
        # norm screening of the block products at several thresholds (tau = 1e-6); accuracy
        # from ||[F, D]||_F
        D, _ = snf.purify_bsr(rp, ci, va, m.n, "snf_varmu", trunc_tau=1e-6, want_log=False,
                              screen_tau=1e-7, **kw)
        del D
        for scheme in ("snf_varmu", "sp2"):
            for tau_s in (0.0, 1e-9, 1e-8, 1e-7, 1e-6):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                D, r = snf.purify_bsr(rp, ci, va, m.n, scheme, trunc_tau=1e-6,
                                      screen_tau=tau_s, **kw)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3
                comm = _bsr_commutator((rp, ci, va), D, m.n)
                print(json.dumps(dict(scheme=scheme, screen_tau=tau_s, ms=round(ms, 1),
                                      product_ms=round(r["product_ms"], 1),
                                      products=r["products"], status=r["status"],
                                      e=r["idem_err"], trace_err=r["trace_err"],
                                      commutator=comm,
                                      blocks_per_row=round(r["blocks"] / m.nb, 1))),
                      flush=True)
                del D
    res = {}
    for scheme in ("snf_varmu", "sp2"):
        for _ in range(args.warmup):
            snf.purify_bsr(rp, ci, va, m.n, scheme, trunc_tau=1e-6, want_log=False, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = max(1, args.steps)
        for _ in range(steps):
            D, r = snf.purify_bsr(rp, ci, va, m.n, scheme, trunc_tau=1e-6, want_log=True, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[scheme] = dict(ms=round(ms, 1), products=r["products"], status=r["status"],
                           idem_err=r["idem_err"], trace_err=r["trace_err"],
                           blocks_D=r["blocks"], blocks_per_row=round(r["blocks"] / m.nb, 1),
                           product_ms=round(r["product_ms"], 1),
                           useful_tflops=round(r["flops"] / (r["product_ms"] * 1e-3) / 1e12, 2),
                           blocks_per_row_by_iterate=[round(x["phase"] / m.nb, 1)
                                                      for x in r["log"]],
                           branches=r["branches"])
        res[scheme]["commutator"] = _bsr_commutator((rp, ci, va), D, m.n)
        del D
    # the same solves with the block products norm-screened at 1e-8 (100x below the
    # truncation threshold): time, and accuracy through ||[F, D]||_F against the unscreened
    screened = {}
    for scheme in (() if args.no_screened else ("snf_varmu", "sp2")):
        tau_s = 1e-8
        snf.purify_bsr(rp, ci, va, m.n, scheme, trunc_tau=1e-6, screen_tau=tau_s,
                       want_log=False, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = max(1, args.steps)
        for _ in range(steps):
            D, r = snf.purify_bsr(rp, ci, va, m.n, scheme, trunc_tau=1e-6, screen_tau=tau_s,
                                  want_log=False, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        screened[scheme] = dict(screen_tau=tau_s, ms=round(ms, 1), products=r["products"],
                                status=r["status"], idem_err=r["idem_err"],
                                trace_err=r["trace_err"],
                                commutator=_bsr_commutator((rp, ci, va), D, m.n),
                                speedup_vs_unscreened=round(res[scheme]["ms"] / ms, 3))
        del D
    s = res["snf_varmu"]
    line = _base_line("time-to-solution ms at the truncation floor (block-sparse), SnF vs SP2",
                      s["ms"], "ms", args, False, "f32",
                      {"workload": "BSR two-orbital lattice 32x32x32 sites, n=65536, 32x32 "
                                   "blocks (4x2x2-site bricks, Morton order), tau=1e-6, half "
                                   "filling", "scheme": "snf_varmu"})
    line["ms_per_step"] = s["ms"]
    line["schemes"] = res
    line["speedup_vs_sp2"] = round(res["sp2"]["ms"] / s["ms"], 3)
    line["norm_screened"] = screened
    line["roofline"] = dict(bound="mfma", achieved=s["useful_tflops"], peak=157.3,
                            unit="TFLOP/s", frac=round(s["useful_tflops"] / 157.3, 4),
                            traffic=None, kernel="bsr_product_kernel (f32 MFMA super-tiles)",
                            note="achieved = 2*32^3 flops per stored-block triple (I,K,J), "
                                 "I<=J, over the summed numeric-kernel time")
    bt = load_bsr_traffic()
    if bt is not None:
        per_launch = bt["product_bytes"] / bt["product_launches"]
        line["roofline"]["traffic"] = per_launch
        line["hbm"] = dict(kernel="bsr_product_kernel", achieved_tbs=round(
            bt["product_bytes"] / (bt["product_ms"] * 1e-3) / 1e12, 2), peak_tbs=8.0,
            frac=round(bt["product_bytes"] / (bt["product_ms"] * 1e-3) / 8e12, 3),
            note="FETCH_SIZE + WRITE_SIZE of the product kernel over both solves (rocprofv3 "
                 "counter runs, copy-calibrated), over its summed time")
    line["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        # the dense block-masked FP64 oracle cannot hold n = 65536 (34 GB per matrix, hours
        # per product): timed on the same lattice recipe at 16x16x8 sites (n = 4096) for the
        # same number of iterations, scaled by the n^3 of its dense products
        from oracle import dense
        ms, hs = H.lattice_bsr((16, 16, 8), seed=3, dtype=np.float64)
        Fs = ms.to_dense()
        t0 = time.perf_counter()
        dense.purify(Fs, "snf_varmu", lambda_min=hs.lambda_min, lambda_max=hs.lambda_max,
                     n_occ=hs.n_occ, homo=hs.homo, lumo=hs.lumo, tol=0.0,
                     max_iter=s["products"] - 1, mask=dense.block_truncation_mask(32, 1e-6))
        dt = time.perf_counter() - t0
        scale = (m.n / ms.n) ** 3
        line["cpu_baseline"] = dict(
            value=round(dt * 1e3 * scale, 0), unit="ms", cores=int(_blas_threads()),
            kind="oracle",
            sample=f"dense block-masked FP64 oracle, same lattice recipe at 16x16x8 sites "
                   f"(n={ms.n}), {s['products'] - 1} iterations: {dt:.1f} s, scaled by "
                   f"(65536/{ms.n})^3 = {scale:.0f}")
    return line


def run_serve(args):
    """512 requests: n log-uniform in [64, 2048], gap log-uniform in [1e-3, 1e-1],
    N_occ = n/2 (1 +- 0.1), FP32 products + FP64 refinement, SnF varying-mu; a closed-loop
    pass measures saturated throughput, then Poisson arrivals at 0.8 of it."""
    import numpy as np
    import torch
    from paper_1101_0265_amd import hamiltonians as H
    from paper_1101_0265_amd import snf
    count = 512
    trace = H.serving_trace(count=count, rate_per_s=1.0, seed=5)
    mats = [H.request_hamiltonian_torch(r, device="cuda:0", keep_on_device=True)
            for r in trace]
    outs = [torch.empty_like(h.F) for h in mats]
    torch.cuda.synchronize()

    def kw(h):
        return dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ,
                    homo=h.homo, lumo=h.lumo, tol=1e-8, max_iter=120, gap_switch=0.0)

    budget = 24 << 30
    flops = 0.0
    flops64 = flops32 = 0.0
    with snf.Server(budget, max_slots=args.serve_slots) as sv:
        # warm-up on a few requests
        for h, o in list(zip(mats, outs))[:args.warmup * 4]:
            sv.wait(sv.submit_device(h.F, "snf_varmu", "fp32_ref64", out=o, **kw(h)))
        t0 = time.perf_counter()
        tickets = [sv.submit_device(h.F, "snf_varmu", "fp32_ref64", out=o, **kw(h))
                   for h, o in zip(mats, outs)]
        for t, h in zip(tickets, mats):
            _, r = sv.wait(t)
            flops += r["flops"]
            per = float(h.n) * h.n * (h.n + 1.0)
            flops64 += r["products_fp64"] * per
            flops32 += r["products_lowp"] * per
        closed_s = time.perf_counter() - t0
    closed_rate = count / closed_s
    # the same closed-loop pass through host buffers (PCIe-inclusive, for context)
    host_F = [h.F.cpu().numpy() for h in mats[:128]]
    with snf.Server(budget, max_slots=args.serve_slots) as sv:
        t0 = time.perf_counter()
        tickets = [sv.submit(F, "snf_varmu", "fp32_ref64", **kw(h))
                   for F, h in zip(host_F, mats[:128])]
        for t in tickets:
            sv.wait(t)
        host_rate = len(host_F) / (time.perf_counter() - t0)
    del host_F
    rate = 0.8 * closed_rate
    gaps = np.random.default_rng(55).exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps)
    lat, statuses = [], []
    with snf.Server(budget, max_slots=args.serve_slots) as sv:
        tickets = []
        t0 = time.perf_counter()
        for h, o, ta in zip(mats, outs, arrivals):
            while time.perf_counter() - t0 < ta:
                time.sleep(5e-5)
            tickets.append(sv.submit_device(h.F, "snf_varmu", "fp32_ref64", out=o, **kw(h)))
        for t in tickets:
            _, r = sv.wait(t)
            statuses.append(r["status"])
            lat.append(sv.timing(t)[2])
        open_s = time.perf_counter() - t0
    lat = np.array(lat)
    line = _base_line("solves/s, continuous batching (512 requests, FP32 + FP64 refinement)",
                      round(count / open_s, 2), "solves/s", args, True, "f32+f64",
                      {"workload": "serving: 512 requests, n log-uniform [64,2048], gap "
                                   "log-uniform [1e-3,1e-1], N_occ=n/2(1+-0.1), Haar Q per "
                                   "request, SnF varying-mu, fp32_ref64; matrices resident "
                                   "in HBM (device submit)",
                       "arrival_rate_per_s": round(rate, 2), "hbm_budget_gb": budget >> 30,
                       "max_slots": args.serve_slots})
    line["latency_ms"] = dict(p50=round(float(np.percentile(lat, 50)), 2),
                              p99=round(float(np.percentile(lat, 99)), 2),
                              mean=round(float(lat.mean()), 2))
    line["closed_loop_solves_per_s"] = round(closed_rate, 2)
    line["closed_loop_host_buffers_solves_per_s"] = round(host_rate, 2)
    line["closed_loop_tflops"] = round(flops / closed_s / 1e12, 2)
    # the mixed FP32/FP64 work against the time it would take at both MFMA peaks
    blend = (flops64 + flops32) / (flops64 / 78.6e12 + flops32 / 157.3e12) / 1e12
    achieved = (flops64 + flops32) / closed_s / 1e12
    line["roofline"] = dict(bound="mfma", achieved=round(achieved, 2), peak=round(blend, 1),
                            unit="TFLOP/s", frac=round(achieved / blend, 4), traffic=None,
                            kernel="grouped_product_kernel (f64 and f32, closed loop)",
                            note=f"peak = the FP64 (78.6) and FP32 (157.3) MFMA peaks weighted "
                                 f"by this run's work: {flops64 / 1e12:.1f} TFLOP in FP64, "
                                 f"{flops32 / 1e12:.1f} in FP32; achieved over the closed-loop "
                                 f"wall time")
    line["statuses"] = {s_: statuses.count(s_) for s_ in set(statuses)}
    # oracle on a bounded sample of the same trace: every 8th request, so the sample keeps
    # the trace's mix of orders (the large ones dominate the time, as on the GPU)
    from oracle import dense
    sample = [(mats[i], trace[i]) for i in range(0, count, 8)]
    sample_F = [h.F.cpu().numpy() for h, _ in sample]
    t0 = time.perf_counter()
    for (h, _), F in zip(sample, sample_F):
        dense.purify(F, "snf_varmu", **{k: v for k, v in kw(h).items() if k != "gap_switch"})
    cpu_s = time.perf_counter() - t0
    ns = [r.n for _, r in sample]
    line["cpu_baseline"] = dict(value=round(len(sample) / cpu_s, 2), unit="solves/s",
                                cores=int(_blas_threads()), kind="oracle",
                                sample=f"every 8th request of the trace ({len(sample)} "
                                       f"requests, n {min(ns)}..{max(ns)}; FP64 numpy, one "
                                       f"after another): {cpu_s:.1f} s")
    return line


SUB_KEYS = ("metric", "value", "unit", "ms_per_step", "higher_is_better", "dtype", "config",
            "speedup_vs_sp2", "latency_ms", "closed_loop_solves_per_s", "roofline",
            "roofline_fp32", "roofline_bf16", "hbm", "cpu_baseline", "norm_screened", "runs",
            "schemes")


def other_workloads(args):
    """The other four workloads, each as a compact object with its own roofline and CPU
    baseline (fewer timed repetitions than their own --workload lines)."""
    import types
    import torch
    sub_args = types.SimpleNamespace(**vars(args))
    sub_args.steps = max(1, min(args.steps, 2))
    sub_args.warmup = 1
    sub_args.compact = True
    out = {}
    for name, fn in (("n256_gap0.05", run_small), ("n8192_gap1e-3", run_precision),
                     ("bsr_lattice_n65536", run_bsr), ("serve_512", run_serve)):
        t0 = time.perf_counter()
        line = fn(sub_args)
        torch.cuda.synchronize()
        sub = {k: line[k] for k in SUB_KEYS if k in line}
        sub["wall_s"] = round(time.perf_counter() - t0, 1)
        out[name] = sub
        print(f"# {name}: {sub['value']} {sub['unit']} ({sub['wall_s']} s)", file=sys.stderr,
              flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="dense",
                    choices=["dense", "small", "bsr", "serve", "precision", "bounds",
                             "fixmu"],
                    help="dense: n=4096 lattice (default line); small: n=256 gap-0.05 latency "
                         "of all five schemes; bsr: block-sparse 32^3-site lattice n=65536; "
                         "serve: 512-request continuous-batching trace; precision: n=8192 "
                         "FP64 vs FP32/BF16 products; bounds: device-estimated bounds; fixmu: "
                         "fixed-mu schemes incl. P_{i,j} with mu off-centre, n=4096")
    ap.add_argument("--bsr-sweep", action="store_true",
                    help="with --workload bsr: one solve per (scheme, truncation threshold) of "
                         "the sweep, one JSON line each")
    ap.add_argument("--serve-slots", type=int, default=256,
                    help="serving workload: requests in flight at most")
    ap.add_argument("--no-screened", action="store_true",
                    help="block-sparse workload: only the unscreened solves (for counter runs "
                         "whose per-launch figures belong to the headline solves)")
    ap.add_argument("--bsr-screen", action="store_true",
                    help="block-sparse workload: also run norm-screened products at several "
                         "thresholds, with ||[F, D]||_F estimates")
    ap.add_argument("--bsr-fixmu", action="store_true",
                    help="block-sparse workload: Algorithm 1 beside Algorithm 2 and SP2")
    ap.add_argument("--bsr-ec", action="store_true",
                    help="block-sparse workload: also run fixed-threshold and error-controlled "
                         "truncation at several budgets, with ||[F, D]||_F estimates")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="default workload: leave out the compact objects of the other four "
                         "workloads")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="for hardware-counter runs: a plain 512 MiB device copy (counter "
                         "calibration), then three stand-alone products X.X: the workload's "
                         "X_0 at n=4096, or a seeded symmetric matrix of order --probe-n")
    ap.add_argument("--probe-n", type=int, default=4096)
    ap.add_argument("--probe-precision", default="fp64",
                    choices=["fp64", "fp32", "bf16_ref64"])
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the method's "
              "multi-GPU layout is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1101_0265_amd import hamiltonians as H
    from paper_1101_0265_amd import snf

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    snf.lib()
    dev = torch.device("cuda:0")
    if args.workload != "dense":
        line = {"small": run_small, "bsr": run_bsr, "serve": run_serve,
                "precision": run_precision, "bounds": run_bounds,
                "fixmu": run_fixmu}[args.workload](args)
        print(json.dumps(line), flush=True)
        return
    h = H.lattice_hamiltonian(LATTICE, seed=2)
    n = h.n
    F = torch.tensor(h.F, device=dev)
    D = torch.empty_like(F)
    kw = dict(lambda_min=h.lambda_min, lambda_max=h.lambda_max, n_occ=h.n_occ, homo=h.homo,
              lumo=h.lumo, mu=h.mu, xi=h.xi, tol=TOL, max_iter=200)

    if args.traffic_probe:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        if args.probe_n == n:
            lmax, lmin = h.lambda_max, h.lambda_min
            X0 = (lmax * torch.eye(n, dtype=torch.float64, device=dev) - F) / (lmax - lmin)
        else:   # a seeded symmetric matrix of the requested order (timing does not depend on
                # the values)
            g = torch.Generator(device=dev)
            g.manual_seed(8)
            Z = torch.randn(args.probe_n, args.probe_n, generator=g, device=dev,
                            dtype=torch.float64)
            X0 = (Z + Z.T) / (2.0 * math.sqrt(args.probe_n))
            del Z
        kms = []
        for _ in range(3):
            kms.append(snf.step_dense(X0, X0, 1.0, 0.0, 0.0, args.probe_precision)[2])
        torch.cuda.synchronize()
        print(json.dumps({"traffic_probe": True, "copy_bytes": src.numel() * 8,
                          "n": args.probe_n, "precision": args.probe_precision,
                          "kernel_ms": kms, "kernel_source_hash": kernel_source_hash()}),
              flush=True)
        return

    def solve(scheme, flags=0):
        _, r = snf.purify_dense(F, scheme, out=D, want_log=False, flags=flags, **kw)
        if r["status"] != "ok":
            raise RuntimeError(f"{scheme}: {r['status']}")
        return r

    for _ in range(args.warmup):
        solve("snf_varmu")
        solve("sp2")

    def timed(scheme):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = [solve(scheme, flags=snf.FLAG_TIME_PRODUCTS) for _ in range(args.steps)]
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps, rs

    snf_ms, snf_rs = timed("snf_varmu")
    sp2_ms, sp2_rs = timed("sp2")

    # FP32 products after the X-space gap reaches 0.5, FP64 refinement to the same tol
    def solve_mixed():
        _, r = snf.purify_dense(F, "snf_varmu", "fp32_ref64", out=D, want_log=False,
                                gap_switch=0.5, **kw)
        if r["status"] != "ok":
            raise RuntimeError(f"fp32_ref64: {r['status']}")
        return r
    solve_mixed()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mixed_r = solve_mixed()
    torch.cuda.synchronize()
    mixed_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    D_mixed = D.clone()
    solve("snf_varmu")
    mixed_err = float(torch.linalg.norm(D_mixed - D))

    flops_per_product = float(n) * n * (n + 1)
    prod_ms = sum(r["product_ms"] for r in snf_rs + sp2_rs)
    prods = sum(r["products"] for r in snf_rs + sp2_rs)
    avg_launch_ms = prod_ms / prods
    achieved = flops_per_product / (avg_launch_ms * 1e-3) / 1e12
    traffic = load_traffic()
    roofline = dict(bound="mfma", achieved=round(achieved, 2), peak=PEAK_FP64_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / PEAK_FP64_TFLOPS, 4),
                    traffic=traffic, kernel="product_f64_kernel (f64 MFMA, 128x128 tiles)",
                    avg_launch_ms=round(avg_launch_ms, 4),
                    flops_per_launch=flops_per_product)
    # HBM bytes an ideal product must move: read X (operand) once, write X_new, read the
    # linear term X again in the epilogue: 3 n^2 * 8 B.
    algo_bytes = 3.0 * n * n * 8
    line = {
        "metric": METRIC,
        "value": round(snf_ms, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(snf_ms, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "dense FP64 two-orbital lattice 16x16x8 sites, n=4096, "
                               "half filling, tol 1e-8",
                   "scheme": "snf_varmu", "n": n, "n_occ": h.n_occ, "tol": TOL,
                   "gap": round(h.lumo - h.homo, 6)},
        "sp2_ms": round(sp2_ms, 3),
        "speedup_vs_sp2": round(sp2_ms / snf_ms, 3),
        "products": {"snf_varmu": snf_rs[0]["products"], "sp2": sp2_rs[0]["products"]},
        "xx_tflops_fp64": round(achieved, 2),
        "xx_algorithmic_gbps": round(algo_bytes / (avg_launch_ms * 1e-3) / 1e9, 1),
        "fp32_ref64": {"ms": round(mixed_ms, 3), "products_fp32": mixed_r["products_lowp"],
                       "products_fp64": mixed_r["products_fp64"],
                       "idem_err": mixed_r["idem_err"],
                       "dist_to_fp64_D_frobenius": mixed_err},
        "idem_err": snf_rs[0]["idem_err"],
        "trace_err": snf_rs[0]["trace_err"],
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(h, kw)
    if not args.no_other_workloads:
        del F, D
        torch.cuda.empty_cache()
        line["workloads"] = other_workloads(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
