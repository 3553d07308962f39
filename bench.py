"""Benchmark: quasi-Newton iterations per second and time-to-tolerance at 3D 511^3.

Workload: -div((1+u^2) grad u) = f on (0,1)^3, homogeneous Dirichlet data,
511^3 interior nodes (1.33e8 unknowns), f manufactured from
u = A sin(pi x) sin(pi y) sin(pi z) with the seeded amplitude A (seed 0), U_0 = 0.
Inputs are synthetic and resident in HBM before any timed region.

A step is one full quasi-Newton iteration of the hot path: the fused
residual/nonlinearity/reduction pass, the on-device shift rule, the three
forward mode products (spectral divide fused into the last), and the three
inverse mode products (U -= dU fused into the last).  `value` is FP64
iterations per second over exactly --steps steps, timed with a device
synchronisation on both sides.  Extra fields report time-to-tolerance (relres
1e-10) in FP64 and in the reduced-precision transform forms, the roofline of
the dominant kernel from HIP events recorded around every launch inside the
timed region, and the CPU oracle timed on a bounded sample.
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from paper_2502_03611_amd import Solver  # noqa: E402

METRIC = "time-to-tol & iters/s at 3D 511^3, FP64 vs mixed+learned guess; % MFMA/HBM peak"
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch (read, write) from rocprofv3 FETCH_SIZE / WRITE_SIZE at
# 511^3, the read counter scaled x2.0 and the write counter x1.0 (both
# calibrated on a plain 1 GiB device copy), keyed by kernel.  Each figure is
# valid only while the source file it was taken on is unchanged.
TRAFFIC_SOURCES = {"fold": ("paper_2502_03611_amd/csrc/qn_gemm_fold.hip", "0bf9f6298fde0112"),
                   "pointwise": ("paper_2502_03611_amd/csrc/qn_pointwise.hip", "1f8af7022b255738"),
                   "bf16": ("paper_2502_03611_amd/csrc/qn_gemm_bf16.hip", "37c82a36bc9257ff")}
TRAFFIC = {"k_fold_right_fwd<double,64,128,0>": ("fold", 1.4620e+09, 1.0737e+09),
           "k_fold_left_fwd2<double,64,64,EPI_STORE,0>": ("fold", 1.4551e+09, 1.0737e+09),
           "k_fold_left_fwd<double,128,128,EPI_DIVIDE,0>": ("fold", 1.2608e+09, 1.0737e+09),
           "k_fold_left_inv<double,64,64,0>": ("fold", 1.3845e+09, 1.0716e+09),
           "k_fold_right_inv<double,64,64,EPI_SUB_DENSE,0>": ("fold", 2.5069e+09, 1.0762e+09),
           "k_residual<QUASILIN,double>": ("pointwise", 2.3923e+09, 1.0738e+09),
           "k_gemm_right_bf<2,128,128,EPI_STORE,false,2>": ("bf16", 5.6274e+08, 7.5118e+08),
           "k_gemm_left_bf<2,128,128,EPI_STORE,false,2>": ("bf16", 5.5471e+08, 5.3793e+08),
           "k_gemm_left_bf<2,128,128,EPI_DIVIDE,false,1>": ("bf16", 5.6746e+08, 5.3688e+08),
           "k_gemm_left_bf<2,128,128,EPI_STORE,true,0>": ("bf16", 5.7217e+08, 5.3693e+08),
           "k_gemm_right_bf<2,64,128,EPI_SUB_DENSE,true,0>": ("bf16", 1.6730e+09, 1.1238e+09)}


def traffic_if_current(kernel, n):
    """Measured HBM bytes per launch of `kernel` (name with its tile) at 511^3,
    or None when the workload or tile differs or its source changed since the
    counters were taken."""
    import hashlib
    if n != 511 or kernel not in TRAFFIC:
        return None
    src, rd, wr = TRAFFIC[kernel]
    path, sha_ref = TRAFFIC_SOURCES[src]
    with open(os.path.join(ROOT, path), "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()[:16]
    return rd + wr if sha == sha_ref else None


def stream_reference(n):
    """Device streaming rate for the residual's access mix (read two FP64
    fields, write one), measured with PyTorch's own elementwise add on fields
    of the same size: the practical ceiling the residual is compared with."""
    a = torch.ones(n ** 3, dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    for _ in range(5):
        torch.add(a, b, out=c)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(20):
        torch.add(a, b, out=c)
    e.record()
    e.synchronize()
    ms = s.elapsed_time(e) / 20
    del a, b, c
    return {"kernel": "torch.add(U, F, out=R), FP64, n^3 points", "avg_launch_ms": round(ms, 4),
            "achieved": round(24.0 * n ** 3 / (ms * 1e-3) / 1e9, 1), "unit": "GB/s"}


def library_gemm_reference():
    """Matrix-core rate the vendor GEMM library reaches on this device: one
    square 8192^3 product through torch.matmul (hipBLASLt / rocBLAS) in FP64
    and in FP32, 2 n^3 flops each.  Context for the mode-product kernels,
    whose roofline fraction stays against the published peak."""
    out = {}
    n = 8192
    for name, dt, peak in (("fp64", torch.float64, PEAK_FP64_TFLOPS),
                           ("fp32", torch.float32, PEAK_FP32_TFLOPS)):
        a = torch.rand((n, n), dtype=dt, device="cuda")
        b = torch.rand((n, n), dtype=dt, device="cuda")
        c = torch.empty((n, n), dtype=dt, device="cuda")
        for _ in range(2):
            torch.matmul(a, b, out=c)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(5):
            torch.matmul(a, b, out=c)
        e.record()
        e.synchronize()
        ms = s.elapsed_time(e) / 5
        tf = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
        out[name] = {"avg_ms": round(ms, 3), "tflops": round(tf, 1), "frac_of_peak": round(tf / peak, 3)}
        del a, b, c
    torch.cuda.empty_cache()
    return {"kernel": "torch.matmul, 8192 x 8192 x 8192", **out}


def mfma_probe():
    """Dense rates of register-only MFMA chains (qn_probe_mfma) in TFLOP/s,
    beside the published peaks: a lower bound of the device's matrix-core
    ceiling (the compiler moves the accumulators between register files every
    four rounds; the vendor GEMM reference can exceed it)."""
    from paper_2502_03611_amd._binding import probe_mfma
    out = {}
    for prec, key, peak in (("fp64", "fp64", PEAK_FP64_TFLOPS), ("fp32", "fp32", PEAK_FP32_TFLOPS),
                            ("bf16x3", "bf16", PEAK_BF16_TFLOPS)):
        v = probe_mfma(prec)
        out[key] = {"tflops": round(v, 1), "frac_of_published": round(v / peak, 3)}
    return out


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def solve_to_tol(shape, U, F, u_ex, precisions, runs, u64=None):
    """Per precision: a fresh solver (autotuned, one untimed step), then `runs`
    full solves from U_0 = 0 to relres 1e-10; the median time, the iteration
    count, the error against the exact solution and (not FP64) the relative
    L2 difference from the FP64 result `u64` (the FP64 run sets it when
    listed first).  Returns (records, u64)."""
    out = {}
    for prec in precisions:
        s = Solver(shape, "quasilinear", beta=0.0, precision=prec)
        s.autotune()
        U.zero_()
        s.iterate(U, F, rtol=0.0, max_iter=1)  # untimed warm-up of this context
        times = []
        for _ in range(runs):  # median of several full solves from U_0 = 0
            U.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = s.iterate(U, F, rtol=1e-10, max_iter=400)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        tt = float(np.median(times))
        Uh = U[0].cpu().numpy()
        rec = {"status": st["status"], "iters": st["iters"], "time_to_tol_s": round(tt, 4),
               "runs_s": [round(r, 4) for r in times],
               "iters_per_s": round(st["iters"] / tt, 2), "relres": st["relres"],
               "max_err_vs_exact": float(np.abs(Uh - u_ex).max())}
        if prec == "fp64":
            u64 = Uh
        elif u64 is not None:
            rec["rel_l2_vs_fp64"] = float(np.linalg.norm(Uh - u64) / np.linalg.norm(u64))
        out[prec] = rec
        s.close()
    return out, u64


def mixed_steps(shape, U, F, steps, precisions=("fp32", "bf16x3")):
    """Per reduced-precision form: `steps` timed quasi-Newton steps at n^3 with
    HIP events around every launch (autotuned tiles, one untimed step first).
    Per launch key the average time; the mode products against their roofline:
    FP32 on the folded count (2 n^2 (ne^2 + no^2) flops per product) against
    the FP32 peak, split-bf16 on the dense count times the part products (3
    for bf16x3, 6 for bf16x6) against the bf16 peak, and both against HBM for
    one FP32 read and one FP32 write of the tensor (8 bytes per point)."""
    n = shape[0]
    ne, no = (n + 1) // 2, n // 2
    out = {}
    for prec in precisions:
        s = Solver(shape, "quasilinear", beta=0.0, precision=prec, timing=True)
        s.autotune()
        U.zero_()
        s.iterate(U, F, rtol=0.0, max_iter=1)
        torch.cuda.synchronize()
        s.timing(reset=True)
        U.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.iterate(U, F, rtol=0.0, max_iter=steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tim = s.timing(reset=True)
        rec = {"ms_per_step": round(dt / steps * 1e3, 3), "kernels": {}}
        for k, (cnt, ms) in tim.items():
            if not cnt:
                continue
            avg = ms / cnt
            e = {"launches": cnt, "avg_ms": round(avg, 4)}
            if k.startswith("gemm"):
                if prec == "fp32":
                    fl, peak = 2.0 * n ** 2 * (ne * ne + no * no), PEAK_FP32_TFLOPS
                else:
                    fl = 2.0 * float(n) ** 4 * (3 if prec == "bf16x3" else 6)
                    peak = PEAK_BF16_TFLOPS
                tf = fl / (avg * 1e-3) / 1e12
                gbs = 8.0 * n ** 3 / (avg * 1e-3) / 1e9
                e.update({"tflops": round(tf, 1), "frac_mfma": round(tf / peak, 4),
                          "gbs_fp32_io": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 4)})
            rec["kernels"][k] = e
        rec["tiles"] = s.tiles()
        if prec == "bf16x3":
            # measured HBM bytes of the kept tiles (profiles/traffic_fp64_quasilinear_511.md)
            keys = ["gemm_x", "gemm_yz", "gemm_divide", "gemm_yz_inv", "gemm_yz_inv", "gemm_x_update"]
            # template tails of the 3D path: x product from the input folded along x,
            # output folded along z; z product from the folded input, output folded
            # along y; y product from the folded input with the divide; folded inverses
            tails = {0: "EPI_STORE,false,2", 2: "EPI_STORE,true,0", 3: "EPI_SUB_DENSE,true,0"}
            for key, (kind, axis, tm, tn) in zip(keys, rec["tiles"]):
                form = "k_gemm_right_bf" if kind in (0, 3) else "k_gemm_left_bf"
                tail = tails.get(kind, "EPI_STORE,false,2" if axis == 2 else "EPI_DIVIDE,false,1")
                tr = traffic_if_current(f"{form}<2,{tm},{tn},{tail}>", n)
                e = rec["kernels"].get(key)
                if e is not None and tr is not None:
                    e["traffic"] = tr
                    e["traffic_gbs"] = round(tr / (e["avg_ms"] * 1e-3) / 1e9, 1)
        out[prec] = rec
        s.close()
    return out


def amplitude_sweep(n, runs):
    """Time to tolerance at n^3 for the seeded amplitudes of seeds 0-4 and the
    worst case A = 2 (FP64, FP32 and bf16x3 transforms)."""
    shape = (n, n, n)
    U = torch.zeros((1,) + shape, dtype=torch.float64, device="cuda")
    cases = [(f"seed {k}", synth.amplitude_c3(k)) for k in range(5)] + [("A = 2", 2.0)]
    out = []
    for name, amp in cases:
        log(f"amplitude sweep: {name} (A = {amp:.4f})")
        u_ex, f = synth.manufactured_c3(n, amp)
        F = torch.from_numpy(f[None]).cuda()
        del f
        rec, _ = solve_to_tol(shape, U, F, u_ex, ("fp64", "fp32", "bf16x3"), runs)
        out.append({"case": name, "amplitude": round(amp, 4), **rec})
        del F, u_ex
        torch.cuda.empty_cache()
    del U
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# The paper's own Neumann examples (Section 6.2 Example 1, eq. ex2d1, and
# Section 6.3 Example 1, eq. ex3d1) at the sizes of its mesh tables
# (results2d_space: 200^2 .. 1600^2 nodes; results3D_mesh: 200^3 .. 800^3),
# started like the paper's experiments from the discrete solution plus a
# 0.1-scaled random degree-4 polynomial.  Large inputs are evaluated on the
# device from the same definitions as synth's generators (checked against
# them on the CPU in the tests).


def e4_inputs(n, device="cuda"):
    """synth.neumann_2d on `device`: (u_exact, f), shape (n, n)."""
    x = torch.from_numpy(synth.node_coords(n)).to(device)
    u = torch.cos(2.0 * math.pi * x)[:, None] * torch.cos(math.pi * x)[None, :]
    return u, 5.0 * math.pi ** 2 * u + u ** 3 + u


def e7_inputs(n, a=10.0, b=10.0, device="cuda"):
    """synth.neumann_potential_3d on `device`: (u_exact, f, V), shape (n, n, n)."""
    x = torch.from_numpy(synth.node_coords(n)).to(device)
    c = torch.cos(math.pi * x)
    w = 100.0 * torch.sin(math.pi * x / 4.0) ** 2 + x * x
    u = c[:, None, None] + c[None, :, None] + c[None, None, :]
    v = w[:, None, None] + w[None, :, None] + w[None, None, :]
    f = (math.pi ** 2 + a) * u
    f += b * u ** 3
    f += v * u
    return u, f, v


def perturbation(n, dim, seed, device="cuda", coords=None):
    """synth.polynomial_perturbation on `device` (same coefficients and nodes)."""
    coef = torch.from_numpy(synth.polynomial_coefficients(dim, seed)).to(device)
    x = torch.from_numpy(synth.node_coords(n) if coords is None else coords).to(device)
    powers = torch.stack([x ** e for e in range(coef.shape[0])])  # (degree+1, n)
    pt = powers.t().contiguous()                                   # (n, degree+1)
    if dim == 2:
        yx = pt @ (coef.t().contiguous() @ powers)                 # sum_j y^j sum_i a_ij x^i
    else:
        k = coef.shape[0]
        kyx = torch.stack([pt @ (coef[:, :, kk].t().contiguous() @ powers) for kk in range(k)])
        yx = (pt @ kyx.reshape(k, n * n)).reshape(n, n, n)
    return yx / yx.abs().max()


def neumann_table_row(shape, F, V, u_ex, lin, cub, fixed_beta, seeds, timing=False,
                      rules=("sum", "max")):
    """One size of a mesh table: the discrete solution U* (midpoint iteration
    from the sampled exact solution to relres 1e-12, or 60 iterations at its
    rounding floor),
    then for each seed a timed solve from U* + 0.1 p to relres 1e-10 with the
    midpoint shift (FP64 and FP32 transforms) and with the fixed shift
    `fixed_beta` and with the other shift rules of the tables (`rules`: min +
    max, max, min of the Jacobian diagonal; FP64).  Iterations and seconds:
    mean, std, median."""
    n, dim = shape[0], len(shape)
    s = Solver(shape, "cubic", beta_mode="midpoint", boundary="neumann", lin=lin, cub=cub,
               potential=V)
    s.autotune()
    Ustar = u_ex[None].clone()
    st = s.iterate(Ustar, F, rtol=1e-12, max_iter=60)  # the floor at 1600^2 is ~2e-12
    s.close()
    rec = {"n": n, "unknowns": n ** dim,
           "discrete_solution": {"iters": st["iters"], "relres": st["relres"],
                                 "max_err_vs_exact": float((Ustar[0] - u_ex).abs().max())}}
    U = torch.empty_like(Ustar)
    kernels = None
    configs = [("midpoint_fp64", "midpoint", 0.0, "fp64"),
               ("midpoint_fp32", "midpoint", 0.0, "fp32"),
               (f"beta{fixed_beta:g}_fp64", "fixed", fixed_beta, "fp64")]
    configs += [(f"{r}_fp64", r, 0.0, "fp64") for r in rules]
    for label, mode, beta, prec in configs:
        tm = timing and label == "midpoint_fp64"
        solver = Solver(shape, "cubic", beta=beta, beta_mode=mode, boundary="neumann", lin=lin,
                        cub=cub, potential=V, precision=prec, timing=tm)
        solver.autotune()
        U.copy_(Ustar)
        solver.iterate(U, F, rtol=0.0, max_iter=1)  # untimed warm-up of this context
        if tm:
            torch.cuda.synchronize()
            solver.timing(reset=True)
        iters, times, bad = [], [], 0
        for seed in seeds:
            U.copy_(Ustar)
            U[0].add_(perturbation(n, dim, seed), alpha=0.1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = solver.iterate(U, F, rtol=1e-10, max_iter=500)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            iters.append(st["iters"])
            bad += st["status"] != 0
        if tm:
            kernels = {k: {"launches": v[0], "avg_ms": round(v[1] / max(v[0], 1), 4)}
                       for k, v in solver.timing(reset=True).items() if v[0]}
        solver.close()
        rec[label] = {"iters_mean": round(float(np.mean(iters)), 2),
                      "iters_std": round(float(np.std(iters)), 2),
                      "time_mean_s": round(float(np.mean(times)), 4),
                      "time_std_s": round(float(np.std(times)), 4),
                      "time_median_s": round(float(np.median(times)), 4),
                      "not_converged": bad, "seeds": len(seeds),
                      "max_err_vs_exact": float((U[0] - u_ex).abs().max())}
        log(f"  n={n} {label}: iters {rec[label]['iters_mean']} +- {rec[label]['iters_std']}, "
            f"median {rec[label]['time_median_s']} s")
    if kernels is not None:
        rec["kernels_midpoint_fp64"] = kernels
        if "residual" in kernels:
            # residual pass: read U, F, V on the nodes, write R into the padded transform tensor
            pts = float(n) ** dim
            padded = 1.0
            for t in shape:
                padded *= 2 * (-(-((t + 1) // 2) // 32) * 32)
            r_bytes = 24.0 * pts + 8.0 * padded if V is not None else 16.0 * pts + 8.0 * padded
            gbs = r_bytes / (kernels["residual"]["avg_ms"] * 1e-3) / 1e9
            rec["residual_hbm"] = {"algorithmic_bytes": r_bytes, "achieved_gbs": round(gbs, 1),
                                   "frac": round(gbs / PEAK_HBM_GBS, 4)}
        ne, no = (n + 1) // 2, n // 2
        fl = 2.0 * float(n) ** (dim - 1) * (ne * ne + no * no)
        prods = [k for k in kernels if k.startswith("gemm")]
        tot_ms = sum(kernels[k]["avg_ms"] * kernels[k]["launches"] for k in prods)
        tot_launch = sum(kernels[k]["launches"] for k in prods)
        rec["mode_products_folded_tflops"] = round(fl * tot_launch / (tot_ms * 1e-3) / 1e12, 2)
    return rec


def paper_tables(seeds2d, seeds3d):
    """Rows of Tables results2d_space (eq. ex2d1: lambda = 1, b = 1; midpoint,
    min + max, max, min and beta = 3) and results3D_mesh (eq. ex3d1:
    lambda = b = 10, V; midpoint, min + max, max and beta = 200)."""
    out = {"e4_2d": [], "e7_3d": []}
    for n in (200, 400, 800, 1600):
        log(f"paper table 2D n={n}")
        u_ex, f = e4_inputs(n)
        out["e4_2d"].append(neumann_table_row((n, n), f[None].contiguous(), None, u_ex, 1.0, 1.0,
                                              3.0, range(seeds2d),
                                              rules=("sum", "max", "min")))
        del u_ex, f
    for n, k in ((200, seeds3d), (400, max(seeds3d // 2, 2)), (800, max(seeds3d // 6, 2))):
        log(f"paper table 3D n={n}")
        u_ex, f, v = e7_inputs(n)
        out["e7_3d"].append(neumann_table_row((n, n, n), f[None].contiguous(), v, u_ex, 10.0,
                                              10.0, 200.0, range(k), timing=(n == 800)))
        del u_ex, f, v
        torch.cuda.empty_cache()
    return out


def batched_tables(seeds, sizes=(200, 400, 800, 1600), all_rules=True):
    """The 2D rows of Table results2d_space (eq. ex2d1) with all perturbed
    starts of one size solved together by the batched solver (one instance
    per seed, Neumann data): the midpoint shift with FP64 and FP32 transforms
    and the table's other rules (beta = 3, min + max, max, min; FP64); the
    midpoint FP64 batch against the same starts solved one after another by
    the single-problem solver.
    Seconds: the whole batch, inputs resident in HBM, after an untimed solve
    of the same batch (graph capture, autotuning)."""
    from paper_2502_03611_amd.batched import BatchedSolver
    out = []
    for n in sizes:
        log(f"batched table 2D n={n}, {seeds} starts")
        u_ex, f = e4_inputs(n)
        s = Solver((n, n), "cubic", beta_mode="midpoint", boundary="neumann", length=2.0, lin=1.0)
        s.autotune()
        Ustar = u_ex[None].clone()
        s.iterate(Ustar, f[None].contiguous(), rtol=1e-12, max_iter=60)
        starts = [Ustar[0] + 0.1 * perturbation(n, 2, seed) for seed in range(seeds)]
        rec = {"n": n, "instances": seeds}
        # one after another (the single-problem solver, FP64)
        U1 = torch.empty_like(Ustar)
        F1 = f[None].contiguous()
        U1.copy_(starts[0][None])
        s.iterate(U1, F1, rtol=1e-10, max_iter=500)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        seq_iters = []
        for u0 in starts:
            U1.copy_(u0[None])
            seq_iters.append(s.iterate(U1, F1, rtol=1e-10, max_iter=500)["iters"])
        torch.cuda.synchronize()
        rec["sequential_fp64"] = {"seconds": round(time.perf_counter() - t0, 4),
                                  "iters_mean": round(float(np.mean(seq_iters)), 2)}
        s.close()
        configs = (("midpoint", 0.0, "fp64"), ("midpoint", 0.0, "fp32"), ("fixed", 3.0, "fp64"),
                   ("sum", 0.0, "fp64"), ("max", 0.0, "fp64"), ("min", 0.0, "fp64"))
        for mode, beta, prec in configs if all_rules else configs[:1]:
            label = prec if mode == "midpoint" else f"{mode}{beta:g}_{prec}" if beta else \
                f"{mode}_{prec}"
            b = BatchedSolver([n] * seeds, [1] * seeds, precision=prec, beta_mode=mode, beta=beta,
                              boundary="neumann", length=2.0, lin=1.0)
            U, F = b.pool(), b.pool()
            for i in range(seeds):
                b.view(F, i)[0].copy_(f)
            b.autotune()

            def fill():
                for i, u0 in enumerate(starts):
                    b.view(U, i)[0].copy_(u0)

            fill()
            b.iterate(U, F, rtol=1e-10, max_iter=500, graph_iters=4)  # capture + warm-up
            fill()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            status, res = b.iterate(U, F, rtol=1e-10, max_iter=500, graph_iters=4)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            its = [r["iters"] for r in res]
            err = max(float((b.view(U, i)[0] - u_ex).abs().max()) for i in range(seeds))
            rec[f"batched_{label}"] = {"seconds": round(dt, 4),
                                      "seconds_per_start": round(dt / seeds, 6),
                                      "iters_mean": round(float(np.mean(its)), 2),
                                      "iters_std": round(float(np.std(its)), 2),
                                      "not_converged": sum(r["status"] != 0 for r in res),
                                      "iters_equal_sequential": int(sum(
                                          a == c for a, c in zip(its, seq_iters)))
                                      if mode == "midpoint" else None,
                                      "max_err_vs_exact": err}
            log(f"  n={n} batched {label}: {dt:.4f} s for {seeds} starts "
                f"(sequential midpoint fp64 {rec['sequential_fp64']['seconds']} s), "
                f"iters {rec[f'batched_{label}']['iters_mean']}")
            b.close()
            del U, F, b
            torch.cuda.empty_cache()
        out.append(rec)
        del u_ex, f, Ustar, U1, F1, starts
        torch.cuda.empty_cache()
    return out


def beta_tables(seeds2d, seeds3d):
    """Tables results2d1 (eq. ex2d1 on 50^2 nodes) and results3D (eq. ex3d1 on
    200^3 nodes) of the paper: for each perturbation scale eps in {0.1, 0.2,
    0.5, 1.0} and each shift rule of the table (the midpoint, min + max, max,
    min in 2D, and the fixed shifts), the mean and std of the iterations from
    U* + eps p to relres 1e-10 and the median time per solve (FP64)."""
    out = {}
    for label, n, dim, rules, fixed in (
            ("e4_2d_50", 50, 2, ("midpoint", "sum", "max", "min"), (3.0, 5.0, 7.0, 9.0, 11.0)),
            ("e7_3d_200", 200, 3, ("midpoint", "sum", "max"), (175.0, 200.0, 250.0, 300.0, 350.0))):
        log(f"beta table {label}")
        shape = (n,) * dim
        if dim == 2:
            u_ex, f = e4_inputs(n)
            V, lin, cub = None, 1.0, 1.0
        else:
            u_ex, f, V = e7_inputs(n)
            lin, cub = 10.0, 10.0
        F = f[None].contiguous()
        s = Solver(shape, "cubic", beta_mode="midpoint", boundary="neumann", lin=lin, cub=cub,
                   potential=V)
        s.autotune()
        Ustar = u_ex[None].clone()
        s.iterate(Ustar, F, rtol=1e-12, max_iter=60)
        s.close()
        seeds = seeds2d if dim == 2 else seeds3d
        U = torch.empty_like(Ustar)
        rows = {}
        for rule in rules + tuple(f"beta{b:g}" for b in fixed):
            mode, beta = (rule, 0.0) if not rule.startswith("beta") else ("fixed", float(rule[4:]))
            solver = Solver(shape, "cubic", beta=beta, beta_mode=mode, boundary="neumann", lin=lin,
                            cub=cub, potential=V)
            solver.autotune()
            rows[rule] = {}
            for eps in (0.1, 0.2, 0.5, 1.0):
                iters, times, bad = [], [], 0
                for seed in range(seeds):
                    U.copy_(Ustar)
                    U[0].add_(perturbation(n, dim, seed), alpha=eps)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st = solver.iterate(U, F, rtol=1e-10, max_iter=3000)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                    iters.append(st["iters"])
                    bad += st["status"] != 0
                rows[rule][f"{eps:g}"] = {"iters_mean": round(float(np.mean(iters)), 2),
                                          "iters_std": round(float(np.std(iters)), 2),
                                          "time_median_s": round(float(np.median(times)), 5),
                                          "not_converged": bad}
            solver.close()
            log(f"  {label} {rule}: " + ", ".join(f"eps {e}: {v['iters_mean']}"
                                                 for e, v in rows[rule].items()))
        out[label] = {"n": n, "seeds": seeds, "rows": rows}
        del u_ex, f, F, Ustar, U
        torch.cuda.empty_cache()
    return out


def e5_table(seeds):
    """Table results2D_2 of the paper (Section 6.2 Example 2, eq. 2dex:
    -Lap u - u^2 = -1600 sin(pi x) sin(pi y) on (0, 1)^2, Dirichlet data): the
    stable solution U* from U_0 = 0 (midpoint shift), then timed solves from
    U* + eps p (p on the interior nodes) to relres 1e-10: eps in {0.1, 0.2,
    0.5, 1.0} at 200^2 and eps = 0.1 at 400^2 .. 1600^2; FP64 and FP32
    transforms, midpoint shift."""
    out = []
    for n in (200, 400, 800, 1600):
        log(f"e5 table n={n}")
        shape = (n, n)
        xs = synth.grid_coords(n)
        x = torch.from_numpy(xs).cuda()
        F = (-1600.0 * torch.sin(math.pi * x)[:, None] * torch.sin(math.pi * x)[None, :])[None]
        F = F.contiguous()
        s = Solver(shape, "cubic", beta_mode="midpoint", cub=1e-300, quad=-1.0)
        s.autotune()
        Ustar = torch.zeros_like(F)
        st = s.iterate(Ustar, F, rtol=1e-12, max_iter=100)
        s.close()
        rec = {"n": n, "stable_solution": {"iters_from_zero": st["iters"], "relres": st["relres"],
                                           "min": float(Ustar.min()), "max": float(Ustar.max())}}
        U = torch.empty_like(Ustar)
        for prec in ("fp64", "fp32"):
            solver = Solver(shape, "cubic", beta_mode="midpoint", cub=1e-300, quad=-1.0,
                            precision=prec)
            solver.autotune()
            U.copy_(Ustar)
            solver.iterate(U, F, rtol=0.0, max_iter=1)  # untimed warm-up of this context
            for eps in ((0.1, 0.2, 0.5, 1.0) if n == 200 else (0.1,)):
                iters, times, bad = [], [], 0
                for seed in range(seeds):
                    U.copy_(Ustar)
                    U[0].add_(perturbation(n, 2, seed, coords=xs), alpha=eps)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st = solver.iterate(U, F, rtol=1e-10, max_iter=500)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                    iters.append(st["iters"])
                    bad += st["status"] != 0
                rec[f"eps{eps:g}_{prec}"] = {"iters_mean": round(float(np.mean(iters)), 2),
                                             "iters_std": round(float(np.std(iters)), 2),
                                             "time_median_s": round(float(np.median(times)), 5),
                                             "not_converged": bad, "seeds": seeds}
                log(f"  n={n} eps {eps} {prec}: iters {np.mean(iters):.2f} +- {np.std(iters):.2f}, "
                    f"median {np.median(times):.5f} s")
            solver.close()
        out.append(rec)
        del F, Ustar, U
        torch.cuda.empty_cache()
    return out


def e8_inputs(n, device="cuda"):
    """synth.schrodinger_3d on `device`: (V, u_start), shape (n, n, n)."""
    x = torch.from_numpy(synth.interior_coords(n, -8.0, 8.0)).to(device)
    w = 100.0 * torch.sin(math.pi * x / 4.0) ** 2 + x * x
    g = torch.exp(-0.5 * x * x)
    v = w[:, None, None] + w[None, :, None] + w[None, None, :]
    u = g[:, None, None] * g[None, :, None] * g[None, None, :]
    return v, u


def eigen_table(seeds, max_n=800):
    """Table results3D_2 of the paper (Section 6.3 Example 2, eq. ex3d2:
    alpha = 1600, the lattice-plus-harmonic potential on (-8, 8)^3, Dirichlet
    data) with the midpoint shift: per size the converged pair U* (from the
    Gaussian start to ||R||_M/|lam| <= 1e-11), then timed solves from
    U* + eps p (normalised by the iteration) to 1e-10: eps = 0.1 at 200^3,
    400^3 and 800^3, and eps = 0.2, 0.3 at 200^3; FP64 transforms, and FP32
    transforms at 200^3 and 400^3."""
    rows = []
    plan = [(200, [0.1, 0.2, 0.3], seeds, ("fp64", "fp32")),
            (400, [0.1], max(seeds // 3, 2), ("fp64", "fp32")),
            (800, [0.1], 2, ("fp64",))]
    for n, epss, k, precs in plan:
        if n > max_n:
            continue
        log(f"eigen table n={n}")
        shape = (n, n, n)
        V, u0 = e8_inputs(n)
        coords = synth.interior_coords(n, -8.0, 8.0)
        s = Solver(shape, "cubic", beta_mode="midpoint", length=16.0, cub=1600.0, potential=V)
        s.autotune()
        Ustar = u0[None].clone()
        t0 = time.perf_counter()
        st = s.eigen_iterate(Ustar, rtol=1e-11, max_iter=4000)
        torch.cuda.synchronize()
        rec = {"n": n, "unknowns": n ** 3,
               "converged_pair": {"iters_from_gaussian": st["iters"], "relres": st["relres"],
                                  "lam": st["lam"], "seconds": round(time.perf_counter() - t0, 3)}}
        log(f"  n={n} U*: {st['iters']} iterations, lam {st['lam']:.10f}")
        s.close()
        U = torch.empty_like(Ustar)
        for prec in precs:
            solver = Solver(shape, "cubic", beta_mode="midpoint", length=16.0, cub=1600.0,
                            potential=V, precision=prec)
            solver.autotune()
            U.copy_(Ustar)
            solver.eigen_iterate(U, rtol=0.0, max_iter=1)  # untimed warm-up of this context
            for eps in epss:
                iters, times, lams, bad = [], [], [], 0
                for seed in range(k):
                    U.copy_(Ustar)
                    U[0].add_(perturbation(n, 3, seed, coords=coords), alpha=eps)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st = solver.eigen_iterate(U, rtol=1e-10, max_iter=6000)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                    iters.append(st["iters"])
                    lams.append(st["lam"])
                    bad += st["status"] != 0
                key = f"eps{eps:g}_{prec}"
                rec[key] = {"iters_mean": round(float(np.mean(iters)), 2),
                            "iters_std": round(float(np.std(iters)), 2),
                            "time_mean_s": round(float(np.mean(times)), 4),
                            "time_median_s": round(float(np.median(times)), 4),
                            "lam_spread": float(max(lams) - min(lams)), "lam": lams[0],
                            "not_converged": bad, "seeds": k}
                log(f"  n={n} {key}: iters {rec[key]['iters_mean']} +- {rec[key]['iters_std']}, "
                    f"median {rec[key]['time_median_s']} s, lam {lams[0]:.10f}")
            solver.close()
        rows.append(rec)
        del V, u0, Ustar, U
        torch.cuda.empty_cache()
    return rows


def sem_comparison(n, runs):
    """The same 3D problem, -Lap u + u^3 = f on (0, 1)^3 with Dirichlet data and
    u = 2 sin(pi x) sin(pi y) sin(pi z), on n^3 unknowns discretised by finite
    differences (Section 3.2) and by Q^2 and Q^4 spectral elements (Section
    3.1; the solve kernels are the same, the residual is the banded H kernel):
    setup time, median time to relres 1e-10 from U_0 = 0 (FP64 and FP32
    transforms, midpoint shift), iterations, the nodal error against u, and
    per-kernel HIP-event averages of the FP64 runs."""
    shape = (n, n, n)
    out = {}
    for label, kw in (("fd", {}), ("sem_q2", dict(discretization="sem", sem_order=2)),
                      ("sem_q4", dict(discretization="sem", sem_order=4))):
        for prec in ("fp64", "fp32"):
            t0 = time.perf_counter()
            s = Solver(shape, "cubic", beta_mode="midpoint", precision=prec,
                       timing=prec == "fp64", **kw)
            t_setup = time.perf_counter() - t0
            g = [torch.sin(math.pi * torch.from_numpy(s.nodes(a)).cuda()) for a in range(3)]
            u = 2.0 * g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :]
            F = (3.0 * math.pi ** 2 * u + u ** 3)[None].contiguous()
            s.autotune()
            U = torch.zeros_like(F)
            s.iterate(U, F, rtol=0.0, max_iter=1)  # untimed warm-up of this context
            torch.cuda.synchronize()
            s.timing(reset=True)
            times = []
            for _ in range(runs):
                U.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = s.iterate(U, F, rtol=1e-10, max_iter=200)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            rec = {"setup_s": round(t_setup, 3), "iters": st["iters"], "status": st["status"],
                   "time_to_tol_s": round(float(np.median(times)), 4),
                   "runs_s": [round(t, 4) for t in times],
                   "max_err_vs_exact": float((U[0] - u).abs().max())}
            if prec == "fp64":
                rec["kernels"] = {k: {"launches": v[0], "avg_ms": round(v[1] / max(v[0], 1), 4)}
                                  for k, v in s.timing(reset=True).items() if v[0]}
                r_ms = rec["kernels"]["residual"]["avg_ms"]
                pb = 24.0 * n ** 3  # read U and F, write R (8 B each)
                rec["residual_gbs"] = round(pb / (r_ms * 1e-3) / 1e9, 1)
            log(f"  {label} {prec}: {st['iters']} iterations, {rec['time_to_tol_s']} s, "
                f"max err {rec['max_err_vs_exact']:.3e}, setup {rec['setup_s']} s")
            out[f"{label}_{prec}"] = rec
            s.close()
            del U, F, u, g
            torch.cuda.empty_cache()
    return out


def cpu_baseline(n, amp):
    """The CPU oracle, as it stands, on a bounded sample: one quasi-Newton
    iteration (residual, shift rule, tensor-product solve, residual) at the
    same 511^3 workload.  Returns iterations per second."""
    from threadpoolctl import threadpool_info

    from oracle import qn as oqn

    _, f = synth.manufactured_c3(n, amp)
    log("cpu baseline: one oracle iteration")
    t0 = time.perf_counter()
    oqn.qn_solve(oqn.QUASILINEAR, f[None], rtol=0.0, max_iter=1)
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"value": 1.0 / dt, "unit": "iters/s", "cores": int(threads), "kind": "oracle",
            "sample": f"1 quasi-Newton iteration of the same 511^3 quasi-linear workload "
                      f"(NumPy FP64 oracle, {dt:.1f} s)"}


def cpu_baseline_one_thread(n=127):
    """The same oracle on one host thread (BLAS limited to 1), on a smaller
    bounded sample: one quasi-Newton iteration of the quasi-linear workload at
    n^3 = 127^3 (1/64 of the unknowns).  Returns iterations per second."""
    from threadpoolctl import threadpool_limits

    from oracle import qn as oqn

    _, f = synth.manufactured_c3(n, synth.amplitude_c3(0))
    log(f"cpu baseline: one oracle iteration on one thread at {n}^3")
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oqn.qn_solve(oqn.QUASILINEAR, f[None], rtol=0.0, max_iter=1)
        dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "iters/s", "cores": 1, "kind": "oracle",
            "sample": f"1 quasi-Newton iteration of the quasi-linear workload at {n}^3 "
                      f"(NumPy FP64 oracle, BLAS on one thread, {dt:.1f} s)"}


def bench_batched(count):
    """Batched workload: `count` 2D instances, N drawn from {63, ..., 1023}, even
    instances scalar -Lap u + u^3 = f, odd ones the 2-component system, unit-variance
    GRF sources (length scale 0.1); FP32 transforms, FP64 residual/update, midpoint
    shift, autotuned tiles, hipGraph replay.  Time to 1e-10 for the whole batch."""
    from paper_2502_03611_amd.batched import BatchedSolver

    log(f"batched: generating {count} instances")
    inst = [synth.batched_instance(i) for i in range(count)]
    b = BatchedSolver([d["n"] for d in inst], [d["ncomp"] for d in inst], precision="fp32",
                      beta_mode="midpoint")
    F = b.pool()
    for i, d in enumerate(inst):
        b.fill(F, i, d["f"])
    del inst
    log("batched: autotune")
    t0 = time.perf_counter()
    b.autotune()
    t_tune = time.perf_counter() - t0
    U = b.pool()
    b.iterate(U, F, rtol=1e-10, max_iter=100, graph_iters=4)  # warm-up, graph capture
    U.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status, res = b.iterate(U, F, rtol=1e-10, max_iter=100, graph_iters=4)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # transform work per solve and component: 4 folded mode products of
    # 2 n (ne^2 + no^2) flops each (dense formula: 2 n^3)
    flops = sum(r["iters"] * 8.0 * n * (((n + 1) // 2) ** 2 + (n // 2) ** 2) * c
                for r, n, c in zip(res, b.sizes, b.ncomp))
    dense = sum(r["iters"] * 8.0 * n ** 3 * c for r, n, c in zip(res, b.sizes, b.ncomp))
    pts = sum(n * n * c for n, c in zip(b.sizes, b.ncomp))
    its = np.array([r["iters"] for r in res])
    sc = np.array(b.ncomp) == 1
    return {"instances": count, "unknowns": int(pts), "classes": len(b.classes()),
            "status": status, "all_converged": bool(all(r["status"] == 0 for r in res)),
            "time_to_tol_s": round(dt, 4), "solves_total": int(its.sum()),
            "iters_mean_scalar": round(float(its[sc].mean()), 3),
            "iters_mean_system": round(float(its[~sc].mean()), 3), "iters_max": int(its.max()),
            "transform_tflops_fp32": round(flops / dt / 1e12, 2),
            "transform_dense_equivalent_tflops": round(dense / dt / 1e12, 2),
            "autotune_s": round(t_tune, 2),
            "precision": "fp32 transforms, fp64 residual/update"}


def bench_gray_scott(sizes=(200, 400, 800, 1600), batch_radii=(0.18, 0.19, 0.2, 0.21, 0.22, 0.23,
                                                                 0.24, 0.25)):
    """The steady Gray-Scott system of Section 6.2 (eq. 2dgrayeq; the paper's
    parameters, Neumann data on [0, 1]^2, step size 0.1, midpoint shift, FP64
    transforms) at the sizes of the paper's table: per size one damped solve
    to relres 1e-10 from a centred spot (radius 0.2), which reaches a
    non-trivial steady state; then the same spot of eight radii at the
    smallest size as one batch against one after another."""
    from paper_2502_03611_amd.batched import BatchedSolver

    out = {"params": {"da": 2.5e-4, "ds": 5e-4, "rho": 0.04, "mu": 0.065}, "step": 0.1,
           "start": "spot radius 0.2 (A = 0.25, S = 0.5 inside)", "sizes": []}
    for n in sizes:
        log(f"gray-scott {n}^2")
        s = Solver((n, n), "grayscott", beta_mode="midpoint", boundary="neumann", length=1.0,
                   step=0.1)
        s.autotune()
        u0 = torch.from_numpy(synth.grayscott_spot(n)).cuda()
        F = torch.from_numpy(synth.grayscott_source(n)).cuda()
        U = u0.clone()
        s.iterate(U, F, rtol=0.0, max_iter=2)  # warm-up
        U.copy_(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.iterate(U, F, rtol=1e-10, max_iter=20000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["sizes"].append({"n": n, "status": st["status"], "iters": st["iters"],
                             "time_s": round(dt, 4), "ms_per_iter": round(1e3 * dt / max(st["iters"], 1), 4),
                             "relres": st["relres"], "max_A": float(U[0].max()),
                             "mean_A": float(U[0].mean())})
        s.close()
        del U, u0, F
        torch.cuda.empty_cache()
    n = sizes[0]
    log(f"gray-scott batch of {len(batch_radii)} at {n}^2")
    starts = [synth.grayscott_spot(n, radius=r) for r in batch_radii]
    Fh = synth.grayscott_source(n)
    s = Solver((n, n), "grayscott", beta_mode="midpoint", boundary="neumann", length=1.0, step=0.1)
    s.autotune()
    F1 = torch.from_numpy(Fh).cuda()
    seq_t, seq_it = 0.0, []
    for u0 in starts:
        U = torch.from_numpy(u0).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.iterate(U, F1, rtol=1e-10, max_iter=20000)
        torch.cuda.synchronize()
        seq_t += time.perf_counter() - t0
        seq_it.append(st["iters"])
    b = BatchedSolver([n] * len(starts), [2] * len(starts), precision="fp64", beta_mode="midpoint",
                      boundary="neumann", length=1.0, system="grayscott", step=0.1)
    b.autotune()
    U, F = b.pool(), b.pool()
    for i, u0 in enumerate(starts):
        b.fill(F, i, Fh)
    for rep in range(2):  # the first replay builds the graph
        for i, u0 in enumerate(starts):
            b.fill(U, i, u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status, res = b.iterate(U, F, rtol=1e-10, max_iter=20000, graph_iters=16)
        torch.cuda.synchronize()
        bt = time.perf_counter() - t0
    out["batched"] = {"n": n, "instances": len(starts), "radii": list(batch_radii),
                      "sequential_s": round(seq_t, 4), "sequential_iters": seq_it,
                      "batched_s": round(bt, 4), "batched_iters": [r["iters"] for r in res],
                      "iters_equal_sequential": int(sum(r["iters"] == q for r, q in zip(res, seq_it))),
                      "status": status, "speedup": round(seq_t / bt, 3)}
    return out


def bench_learned(nseeds=500):
    """Learned initial guess on 2D 255^2 -Lap u + u^3 = f with the committed
    trained weights on the held-out seeds: iterations and time to 1e-10 from
    U_0 = 0 and from the learned guess (network in FP16 inference, the guess's
    two solves, the fallback test), FP64 and FP32 transforms, one solve at a
    time; then the same seeds as one batch (FP32 transforms), from U_0 = 0 and
    from the batch of learned guesses."""
    from paper_2502_03611_amd import learned_guess as lg

    if not os.path.exists(lg.WEIGHTS):
        return {"skipped": "no trained weights at " + os.path.relpath(lg.WEIGHTS, ROOT)}
    theta = np.load(lg.WEIGHTS, allow_pickle=False)
    net = lg.Net(255, 255, max_batch=50)
    net.set_params(theta)
    net.set_inference("fp16")
    lg.compare(net, range(10000, 10002))  # warm-up
    log(f"learned guess: {nseeds} held-out seeds, one at a time")
    rows = lg.compare(net, range(10000, 10000 + nseeds))
    outd = {"held_out_seeds": nseeds, "n": 255, "inference": "fp16 fused"}
    for key in ("fp64_zero", "fp64_net", "fp32_zero", "fp32_net"):
        t = np.array([r[key]["t"] for r in rows])
        outd[key] = {"mean_iters": round(float(np.mean([r[key]["iters"] for r in rows])), 3),
                     "mean_time_ms": round(1e3 * float(t.mean()), 3),
                     "median_time_ms": round(1e3 * float(np.median(t)), 3),
                     "all_converged": bool(all(r[key]["status"] == 0 for r in rows)),
                     "max_rel_diff_vs_fp64_zero": float(max(r[key]["rel_diff"] for r in rows))}
        if key.endswith("net"):
            outd[key]["used_net_frac"] = round(float(np.mean([r[key]["used_net"] for r in rows])), 3)
    # medians: single slow solves (host hiccups) move the means
    outd["speedup_fp32_net_vs_fp64_zero"] = round(
        outd["fp64_zero"]["median_time_ms"] / outd["fp32_net"]["median_time_ms"], 3)
    outd["speedup_fp64_net_vs_fp64_zero"] = round(
        outd["fp64_zero"]["median_time_ms"] / outd["fp64_net"]["median_time_ms"], 3)
    log("learned guess: the same seeds as one batch")
    outd["batched"] = lg.compare_batched(net, list(range(10000, 10000 + nseeds)))
    return outd


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=511)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-tol", action="store_true")
    ap.add_argument("--no-mixed-steps", action="store_true",
                    help="skip the timed FP32 / bf16x3 steps with per-kernel times")
    ap.add_argument("--ttt-runs", type=int, default=5,
                    help="timed solves per precision for time to tolerance (median reported)")
    ap.add_argument("--amp-sweep", action="store_true",
                    help="also report time to tolerance for the amplitudes of seeds 0-4 and A = 2")
    ap.add_argument("--paper-tables", action="store_true",
                    help="also run the paper's Neumann mesh tables (2D 200^2-1600^2, "
                         "3D 200^3-800^3, perturbed starts)")
    ap.add_argument("--e5-table", action="store_true",
                    help="also run the paper's table for -Lap u - u^2 = -1600 sin sin (2D, "
                         "Dirichlet; 200^2 .. 1600^2, perturbed stable solution)")
    ap.add_argument("--batched-tables", action="store_true",
                    help="also solve the 2D rows of the paper's Neumann mesh table with all "
                         "perturbed starts of a size in one batch (--table-seeds starts)")
    ap.add_argument("--beta-tables", action="store_true",
                    help="also run the paper's shift-rule tables over perturbation scales "
                         "(eq. ex2d1 at 50^2, eq. ex3d1 at 200^3)")
    ap.add_argument("--table-seeds", type=int, default=20,
                    help="perturbations per 2D size and at 200^3 (fewer at 400^3 and 800^3)")
    ap.add_argument("--eigen-table", action="store_true",
                    help="also run the paper's nonlinear eigenproblem table (eq. ex3d2 at "
                         "200^3, 400^3 and 800^3 from perturbed converged pairs)")
    ap.add_argument("--eigen-max-n", type=int, default=800,
                    help="largest size of the eigenproblem table (200, 400 or 800)")
    ap.add_argument("--eigen-seeds", type=int, default=10,
                    help="perturbations per scale at 200^3 (a third at 400^3, 2 at 800^3)")
    ap.add_argument("--sem", action="store_true",
                    help="also compare finite differences with Q^2 and Q^4 spectral elements on "
                         "the same n^3 unknowns (3D cubic problem, Dirichlet data)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-neumann", action="store_true",
                    help="also solve the 100 perturbed 200^2 Neumann starts (eq. ex2d1) as one "
                         "batch against one after another")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-gray-scott", action="store_true",
                    help="skip the damped Gray-Scott solves (200^2 .. 1600^2 and a batch of 8)")
    ap.add_argument("--batched-count", type=int, default=512)
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (reference kernel "
                         "for scaling HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition of this solver is not built", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        src = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n = args.n
    amp = synth.amplitude_c3(0)
    log(f"generating inputs n={n}")
    u_ex, f = synth.manufactured_c3(n, amp)
    F = torch.from_numpy(f[None]).cuda()
    del f
    shape = (n, n, n)

    log("timed FP64 steps")
    solver = Solver(shape, "quasilinear", beta=0.0, precision="fp64", timing=True)
    U = torch.zeros((1,) + shape, dtype=torch.float64, device="cuda")
    log("autotune mode-product tiles")
    t0 = time.perf_counter()
    solver.autotune()
    t_tune = time.perf_counter() - t0
    tiles = solver.tiles()
    if args.warmup > 0:
        solver.iterate(U, F, rtol=0.0, max_iter=args.warmup)
    torch.cuda.synchronize()
    solver.timing(reset=True)
    U.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = solver.iterate(U, F, rtol=0.0, max_iter=args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert st["iters"] == args.steps, st
    tim = solver.timing(reset=True)
    value = args.steps / dt

    # The mode products run reflection-folded: a product along an axis of n
    # points over L lines does 2 L (ne^2 + no^2) flops (ne = ceil(n/2),
    # no = floor(n/2)), about half the 2 L n^2 of the dense formula.
    ne, no = (n + 1) // 2, n // 2
    flops_per_product = 2.0 * float(n) ** 2 * (ne * ne + no * no)
    dense_flops = 2.0 * float(n) ** 4
    # kernel names per timing key from the tiles in use (launch order: x, y
    # forward, z forward + divide, z and y inverse, x inverse + update)
    def kernel_name(slot, t):
        # kind: 0 x fwd, 1 y/z fwd, 2 y/z inv, 3 x inv; +4 when the tile is
        # paired; + the LDS stage depth when not the kernel's default (the
        # last template argument, 0 for the default)
        kind, _, tm, tn = t
        base, paired, tk = kind & 3, bool(kind & 4), kind & ~7
        if base == 0:
            return f"k_fold_right_fwd<double,{tm},{tn},{tk}>"
        if base == 1:
            epi = "EPI_DIVIDE" if slot == 2 else "EPI_STORE"
            return f"k_fold_left_fwd{'2' if paired else ''}<double,{tm},{tn},{epi},{tk}>"
        if base == 2:
            return f"k_fold_left_inv<double,{tm},{tn},{tk}>"
        return f"k_fold_right_inv<double,{tm},{tn},EPI_SUB_DENSE,{tk}>"
    kname = [kernel_name(i, t) for i, t in enumerate(tiles)]
    names = {"gemm_x": kname[0], "gemm_yz": kname[1], "gemm_divide": kname[2],
             "gemm_yz_inv": kname[3] if kname[3] == kname[4] else kname[3] + " / " + kname[4],
             "gemm_x_update": kname[5]}
    dom = max(names, key=lambda k: tim[k][1])
    launches, tot_ms = tim[dom]
    avg_ms = tot_ms / max(launches, 1)
    achieved = flops_per_product / (avg_ms * 1e-3) / 1e12
    roof = {"bound": "mfma", "kernel": names[dom], "achieved": round(achieved, 3),
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic_if_current(names[dom], n),
            "avg_launch_ms": round(avg_ms, 4), "launches": launches,
            "algorithmic_flops_per_launch": flops_per_product,
            "dense_equivalent_tflops": round(dense_flops / (avg_ms * 1e-3) / 1e12, 3)}
    # the residual pass (HBM-bound): read U and F, write R, 8 bytes each
    rl, rms = tim["residual"]
    r_avg = rms / max(rl, 1)
    r_bytes = 24.0 * n ** 3
    kernels = {k: {"launches": v[0], "avg_ms": round(v[1] / max(v[0], 1), 4)} for k, v in tim.items() if v[0]}
    all_gemm_ms = sum(tim[k][1] for k in names)
    all_gemm_launches = sum(tim[k][0] for k in names)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (manufactured solution, seeded amplitude)",
        "config": {"workload": "3D quasi-linear -div((1+u^2) grad u) = f, 511^3 interior, "
                               "FD Dirichlet, FP64 transforms, U0 = 0",
                   "n": n, "amplitude": amp, "seed": 0},
        "roofline": roof,
        "residual_roofline": {"bound": "hbm", "achieved": round(r_bytes / (r_avg * 1e-3) / 1e9, 1),
                              "peak": PEAK_HBM_GBS, "unit": "GB/s",
                              "frac": round(r_bytes / (r_avg * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                              "traffic": traffic_if_current("k_residual<QUASILIN,double>", n),
                              "avg_launch_ms": round(r_avg, 4),
                              "algorithmic_bytes_per_launch": r_bytes,
                              "stream_reference": stream_reference(n)},
        "library_gemm_reference": library_gemm_reference(),
        "mfma_probe": mfma_probe(),
        "all_mode_products_tflops": round(flops_per_product * all_gemm_launches /
                                          (all_gemm_ms * 1e-3) / 1e12, 3),
        "all_mode_products_dense_equivalent_tflops": round(dense_flops * all_gemm_launches /
                                                           (all_gemm_ms * 1e-3) / 1e12, 3),
        "kernels": kernels,
        "tiles": {"launches": ["x fwd", "y fwd", "z fwd+divide", "z inv", "y inv", "x inv+update"],
                  "kernels": kname, "autotune_s": round(t_tune, 3)},
    }

    if not args.no_mixed_steps:
        log("timed steps with reduced-precision transforms")
        out["mixed_steps"] = mixed_steps(shape, U, F, args.steps)

    if not args.no_time_to_tol:
        solver.close()
        log("time to tolerance: fp64, fp32, bf16x3, bf16x6")
        ttt, _ = solve_to_tol(shape, U, F, u_ex, ("fp64", "fp32", "bf16x3", "bf16x6"),
                              args.ttt_runs)
        out["time_to_tol"] = ttt
        out["speedup_fp32_vs_fp64"] = round(ttt["fp64"]["time_to_tol_s"] / ttt["fp32"]["time_to_tol_s"], 3)
        out["speedup_bf16x3_vs_fp64"] = round(ttt["fp64"]["time_to_tol_s"] / ttt["bf16x3"]["time_to_tol_s"], 3)
        out["speedup_bf16x6_vs_fp64"] = round(ttt["fp64"]["time_to_tol_s"] / ttt["bf16x6"]["time_to_tol_s"], 3)

    solver.close()
    del U, F
    torch.cuda.empty_cache()
    if args.amp_sweep:
        out["amplitude_sweep"] = amplitude_sweep(n, args.ttt_runs)
    if args.paper_tables:
        out["paper_tables"] = paper_tables(args.table_seeds, args.table_seeds)
        torch.cuda.empty_cache()
    if args.batched_tables:
        out["batched_tables"] = batched_tables(args.table_seeds)
        torch.cuda.empty_cache()
    if args.e5_table:
        out["e5_table"] = e5_table(args.table_seeds)
        torch.cuda.empty_cache()
    if args.beta_tables:
        out["beta_tables"] = beta_tables(args.table_seeds, max(args.table_seeds // 3, 2))
        torch.cuda.empty_cache()
    if args.sem:
        out["sem_comparison"] = sem_comparison(n, args.ttt_runs)
        torch.cuda.empty_cache()
    if args.eigen_table:
        out["eigen_table"] = eigen_table(args.eigen_seeds, args.eigen_max_n)
        torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = bench_batched(args.batched_count)
        torch.cuda.empty_cache()
    if args.batched_neumann:
        out["batched_neumann_200"] = batched_tables(100, sizes=(200,), all_rules=False)[0]
        torch.cuda.empty_cache()
    if not args.no_gray_scott:
        out["gray_scott"] = bench_gray_scott()
        torch.cuda.empty_cache()
    if not args.no_learned:
        out["learned_guess"] = bench_learned()
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, amp)
        out["cpu_baseline_one_thread"] = cpu_baseline_one_thread()
    probe64 = out["mfma_probe"]["fp64"]["tflops"]
    out["roofline"]["frac_of_fp64_mfma_probe"] = round(out["roofline"]["achieved"] / probe64, 4)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
