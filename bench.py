#!/usr/bin/env python3
"""Time-to-1e-10 of GMRES-IR (fp32 inner GMRES(50), fp64 refinement) on one MI355X.

Workload (the configuration the comparison of an fp32- and a bf16-stored
Krylov basis against fp64 GMRES is quoted on): the 27-point variable-
coefficient nonsymmetric stencil on a 128^3 grid (N = 2,097,152, 55,742,968
nonzeros; off-diagonals -(1 + 0.3 U[-1,1]) per entry with a skew part of
scale 0.5, row sums 0.05), seed 0, b = A u with u ~ U[-1, 1], x0 = 0, relative
residual tolerance 1e-10, restart m = 50.  One step = one complete solve (fp64
residual, cast, inner cycles of SpMV + CGS2 + Givens, fp64 correction, until
||b - A x|| / ||b|| <= 1e-10).  `value` is the fp32-basis GMRES-IR time; the
bf16-basis GMRES-IR, fp64 GMRES(50) and the learned-parameter variant on the
same GPU and system are timed beside it, and the 2D 1000^2 and 3D 150^3
systems once each as extra keys.  Inputs are resident in HBM before the timed
region.

The CPU oracle solves the same system whole (fp32 GMRES-IR and fp64 GMRES)
on the host's cores: its time is `cpu_baseline` and its solution gives the
fp64 error ||x - x_oracle|| / ||x_oracle|| of every GPU result.

Prints one JSON line.  Options for profiling runs: --no-cpu-baseline,
--no-extras, --no-profile, --copy-calibration (a plain device copy of known
size, for scaling the HBM traffic counters), --only fp32|bf16|fp64 (the
timed solves of one variant only).
"""

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "time-to-1e-10 residual (s), GMRES-IR FP32/BF16 vs FP64 GMRES; SpMV+CGS2 HBM GB/s"
WORKLOAD = "varcoef27_128^3_27pt_seed0"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_varcoef27_128.json")


def kernel_source_hash():
    """sha256 over the library's HIP/C++ sources (names and contents)."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2109_01232_amd", "csrc", "*"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` (a profile category) from the committed
    hardware-counter summary, or None when the sources changed since the
    counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k["traffic_bytes_per_launch"]


def blas_threads():
    try:
        from threadpoolctl import threadpool_info

        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def cpu_oracle(system):
    """The CPU oracle's whole solves of the workload: fp32 GMRES-IR (the GPU
    headline's method) and fp64 GMRES(50), each to 1e-10, timed on the host."""
    from oracle import linalg as L

    t0 = time.perf_counter()
    ir = L.gmres_ir(system.A, system.b, m=50, rtol=1e-10, inner="fp32", check_mode=1)
    t_ir = time.perf_counter() - t0
    t0 = time.perf_counter()
    d64 = L.gmres(system.A, system.b, m=50, rtol=1e-10, check_mode=1)
    t_64 = time.perf_counter() - t0
    return ir, t_ir, d64, t_64


def rel_err(a, b):
    import numpy as np

    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--only", default=None, choices=["fp32", "bf16", "fp64", "dcgs2", "fp64_dcgs2"],
                    help="time only this variant's solves (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-parameter variant")
    ap.add_argument("--no-extras", action="store_true", help="skip the 2D 1000^2 and 3D 150^3 solves")
    ap.add_argument("--spmv-study", action="store_true",
                    help="only time fp64 vs fp32 SpMV over the stencil families (1000 calls, min of 3), "
                         "one JSON line per family")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--max-iters", type=int, default=1_000_000,
                    help="cap on inner iterations of the timed solves (short hardware-counter runs only)")
    ap.add_argument("--suite", action="store_true",
                    help="also time the other workloads and variants (GMRES-FD switch points, block Jacobi, "
                         "polynomial degrees, 3D Laplacian studies, fp32 polynomial in fp64 GMRES); one JSON "
                         "line each, after the main line")
    ap.add_argument("--suite-only", action="store_true")
    ap.add_argument("--suite-case", default=None,
                    help="run only the suite solves whose 'name/inner/basis/restart/degree' label contains this "
                         "text (e.g. 'aniso3d_150_7pt/fp32/fp32/100/0'); for profiling one workload")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU only; --gpus must be 1 "
                                   "(a row-block decomposition over several GPUs is designed, not built)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2109_01232_amd import binding as B
    from paper_2109_01232_amd import problems as P

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    torch.cuda.set_device(0)
    B.lib()

    if args.suite_only:
        suite(args)
        return

    if args.spmv_study:
        spmv_study()
        return

    if args.copy_calibration:
        # plain copy of a known size (256 MiB read + 256 MiB written) for the counter scaling
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").uniform_()
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "launches": 5}), flush=True)
        return

    log("building the 27-point 128^3 system")
    system = P.varcoef27_system(args.seed)
    A = system.A
    # matrix set-up (CSR upload, fp32 copy, sliced copy): reported, not in the solve times
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M = B.Matrix.from_csr(A)
    torch.cuda.synchronize()
    t_matrix = time.perf_counter() - t0
    b = torch.from_numpy(system.b).cuda()
    x = torch.zeros_like(b)
    ws = B.Workspace()
    Asp = A.scipy()
    bnorm = float(np.linalg.norm(system.b))
    m = args.restart

    def timed(p, steps, warmup, roots=None):
        """mean wall time of `steps` solves (after `warmup`), inputs resident;
        returns (seconds, result dict, status, solution on the host)."""
        for _ in range(warmup):
            x.zero_()
            B.gmresir_solve(M, b, x, p, poly_roots=roots, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            st, d, _ = B.gmresir_solve(M, b, x, p, poly_roots=roots, ws=ws)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / max(steps, 1)
        return t, d, st, x.cpu().numpy()

    def describe(t, d, st, xs):
        true = float(np.linalg.norm(system.b - Asp @ xs) / bnorm)
        return {"s": t, "iters": d["iters"], "refinements": d["refinements"], "status": B.status_string(st),
                "rel_resid_true": true, "converged": bool(true <= 1e-10), "sol_err_vs_u": rel_err(xs, system.u)}

    variants = {
        "fp32": B.make_params(restart=m, inner="fp32", basis="fp32", rtol=1e-10, check_mode=1,
                              max_iters=args.max_iters),
        "bf16": B.make_params(restart=m, inner="fp32", basis="bf16", rtol=1e-10, check_mode=1,
                              max_iters=args.max_iters),
        "fp64": B.make_params(restart=m, inner="fp64", rtol=1e-10, check_mode=1, max_iters=args.max_iters),
        # the same fp32 GMRES-IR with the one-reduction CGS2 (second pass delayed one iteration)
        "dcgs2": B.make_params(restart=m, inner="fp32", basis="fp32", rtol=1e-10, check_mode=1,
                               max_iters=args.max_iters, ortho="dcgs2"),
        # and fp64 GMRES(50) with it (the same orthogonalisation on both sides of the comparison)
        "fp64_dcgs2": B.make_params(restart=m, inner="fp64", rtol=1e-10, check_mode=1, max_iters=args.max_iters,
                                    ortho="dcgs2"),
    }
    results, sols = {}, {}
    for name, p in variants.items():
        if args.only and name != args.only:
            continue
        steps = args.steps
        log(f"timed {name} solves: {steps} (warm-up {args.warmup})")
        t, d, st, xs = timed(p, steps, args.warmup)
        results[name] = describe(t, d, st, xs)
        sols[name] = xs
        log(f"{name}: {t:.4f} s/solve iters={d['iters']} resid={results[name]['rel_resid_true']:.3e}")

    head = results.get("fp32") or next(iter(results.values()))
    t_ir = head["s"]
    out = {
        "metric": METRIC,
        "value": t_ir,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_ir * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD if args.seed == 0 else f"varcoef27_128^3_27pt_seed{args.seed}",
            "N": A.n, "nnz": A.nnz, "restart": m, "rtol": 1e-10, "inner": "fp32", "basis": "fp32",
            "check_mode": 1, "x0": "zero", "rhs": "b = A u, u ~ U[-1,1]",
        },
        "iters": head["iters"],
        "refinements": head["refinements"],
        "status": head["status"],
        "converged": head["converged"],
        "rel_resid_true": head["rel_resid_true"],
        "sol_err_vs_u": head["sol_err_vs_u"],
        "matrix_setup_s": t_matrix,
        "matrix_layout": M.layout,
    }
    if "bf16" in results:
        out["bf16_basis"] = results["bf16"]
    if "fp64" in results:
        out["fp64_gmres"] = results["fp64"]
        out["fp64_gmres_s"] = results["fp64"]["s"]
        out["speedup_vs_fp64"] = results["fp64"]["s"] / t_ir
        if "bf16" in results:
            out["bf16_basis"]["speedup_vs_fp64"] = results["fp64"]["s"] / results["bf16"]["s"]
    if "dcgs2" in results:
        out["one_reduction_cgs2"] = results["dcgs2"]
        if "fp64" in results:
            out["one_reduction_cgs2"]["speedup_vs_fp64"] = results["fp64"]["s"] / results["dcgs2"]["s"]
        if "fp32" in results:
            out["one_reduction_cgs2"]["speedup_vs_two_pass_cgs2"] = results["fp32"]["s"] / results["dcgs2"]["s"]
        if "fp64_dcgs2" in results:
            out["one_reduction_cgs2"]["fp64_gmres"] = results["fp64_dcgs2"]
            out["one_reduction_cgs2"]["speedup_vs_fp64_same_orthogonalisation"] = (results["fp64_dcgs2"]["s"] /
                                                                                   results["dcgs2"]["s"])
    if "bf16" in results and "fp32" in results:
        out["bf16_basis"]["s_per_iter_vs_fp32"] = ((results["bf16"]["s"] / results["bf16"]["iters"]) /
                                                   (results["fp32"]["s"] / results["fp32"]["iters"]))

    if not args.only and not args.no_learned and os.path.exists(
            os.path.join(ROOT, "paper_2109_01232_amd", "chooser_weights.json")):
        out["learned"] = learned_variant(M, b, x, ws, system, Asp, args.steps)
        if "fp64" in results:
            out["learned"]["speedup_vs_fp64"] = results["fp64"]["s"] / out["learned"]["s"]

    if not args.no_profile:
        # one more solve with HIP events around every kernel (on the solve's stream)
        pv = "fp32" if not args.only else args.only
        p_prof = B.make_params(restart=m, inner="fp64" if pv.startswith("fp64") else "fp32",
                               basis={"dcgs2": "fp32", "fp64_dcgs2": "fp64"}.get(pv, pv), rtol=1e-10,
                               check_mode=1, profile=1, max_iters=args.max_iters,
                               ortho="dcgs2" if pv.endswith("dcgs2") else "cgs2")
        x.zero_()
        _, d_prof, _ = B.gmresir_solve(M, b, x, p_prof, ws=ws)
        cats = ("spmv_proj", "update_proj", "update_norm")
        dom = max(cats, key=lambda c: d_prof["cat_time_s"][c])
        tt, bb, nl = d_prof["cat_time_s"][dom], d_prof["cat_bytes"][dom], d_prof["cat_launches"][dom]
        achieved = bb / tt / 1e9 if tt > 0 else 0.0
        copy_gbps = device_copy_rate()
        triad_gbps = device_triad_rate()
        traffic = measured_traffic(dom) if (args.seed == 0 and m == 50 and pv == "fp32") else None
        out["roofline"] = {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom, "variant": pv,
            "avg_launch_us": tt / max(nl, 1) * 1e6, "avg_bytes_per_launch": bb / max(nl, 1),
            "launches": nl, "measured_copy_GBps": copy_gbps, "measured_triad_GBps": triad_gbps,
            "bytes_model": "SpMV (4 + 4) nnz + 4 (N + 1) + 2*4 N (x read, w written; 4-byte column indices) + "
                           "4 N per basis column read or written (first CGS2 projection fused)",
        }
        out["breakdown"] = {
            c: {"s": d_prof["cat_time_s"][c], "GBps": (d_prof["cat_bytes"][c] / d_prof["cat_time_s"][c] / 1e9
                                                      if d_prof["cat_time_s"][c] > 0 else 0.0),
                "launches": d_prof["cat_launches"][c]}
            for c in B.CATEGORIES if d_prof["cat_launches"][c] > 0
        }

    if not args.only and not args.no_extras:
        out["extras"] = extras(args, ws, learned=not args.no_learned)

    if not args.no_cpu_baseline and not args.only:
        log("cpu oracle: whole fp32 GMRES-IR and fp64 GMRES solves of the same system")
        ir, t_orc, d64, t_orc64 = cpu_oracle(system)
        x_or = ir.x
        for name, xs in sols.items():
            e = rel_err(xs, x_or)
            if name == "fp32":
                out["sol_err_vs_oracle"] = e
            elif name == "fp64_dcgs2":
                out["one_reduction_cgs2"]["fp64_gmres"]["sol_err_vs_oracle"] = e
            else:
                out[{"bf16": "bf16_basis", "fp64": "fp64_gmres", "dcgs2": "one_reduction_cgs2"}[name]][
                    "sol_err_vs_oracle"] = e
        if "learned" in out and "x" in out["learned"]:
            out["learned"]["sol_err_vs_oracle"] = rel_err(out["learned"].pop("x"), x_or)
        out["oracle_solution"] = {"method": "oracle fp32 GMRES-IR(50), rtol 1e-10", "iters": ir.iters,
                                  "rel_resid": ir.rel_resid, "sol_err_vs_u": rel_err(x_or, system.u),
                                  "fp64_gmres_x_vs_ir_x": rel_err(d64.x, x_or)}
        out["cpu_baseline"] = {
            "value": t_orc,
            "unit": "s",
            "cores": int(blas_threads()),
            "kind": "oracle",
            "sample": (f"the whole solve, not a sample: the oracle's fp32 GMRES-IR(50) on the same 27-point 128^3 "
                       f"system to 1e-10 ({ir.iters} inner iterations, {ir.refinements} refinements); its "
                       f"fp64 GMRES(50) solve took {t_orc64:.1f} s ({d64.iters} iterations)"),
            "fp64_gmres_s": t_orc64,
            "threads_note": "the dense products (V^T w, V h) run on the BLAS thread pool (cores); the scipy SpMV "
                            "and the Givens loop run on one thread",
            "cpu": platform.processor() or platform.machine(),
            "nproc": os.cpu_count(),
        }
    out.get("learned", {}).pop("x", None)

    print(json.dumps(out), flush=True)
    if args.suite:
        suite(args)


def device_copy_rate():
    """A plain 256 MiB device copy on the same GPU, for context beside the published peak."""
    import torch

    src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").uniform_()
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    return 10 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9


def device_triad_rate():
    """STREAM triad a = b + s c over three 512 MiB fp32 arrays (past the 256 MB
    Infinity Cache) on the same GPU: bytes read and written per second."""
    import torch

    b = torch.empty(128 << 20, dtype=torch.float32, device="cuda").uniform_()
    c = torch.empty_like(b).uniform_()
    a = torch.empty_like(b)
    torch.add(b, c, alpha=0.5, out=a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        torch.add(b, c, alpha=0.5, out=a)
    e1.record()
    torch.cuda.synchronize()
    rate = 10 * 3 * b.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b, c
    torch.cuda.empty_cache()
    return rate


def learned_variant(M, b, x, ws, system, Asp, steps):
    """features -> network -> (m, inner cap, polynomial degree), then the
    solve; the timed step includes the features, the network and the
    polynomial set-up."""
    import numpy as np
    import torch

    from paper_2109_01232_amd import binding as B
    from paper_2109_01232_amd import chooser as CH

    net = CH.Chooser.load()

    def step():
        feats = B.gmresir_features(M, b, ws=ws)
        m_c, capm, deg = net.choose(feats)
        roots = B.gmresir_poly_setup(M, deg, seed=12345, ws=ws) if deg > 0 else None
        pc = B.make_params(restart=m_c, inner="fp32", rtol=1e-10, inner_cap=m_c * capm, poly_degree=deg,
                           check_mode=1)
        x.zero_()
        st, d, _ = B.gmresir_solve(M, b, x, pc, poly_roots=roots, ws=ws)
        return (m_c, capm, deg), st, d

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        cfg, st, d = step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / max(steps, 1)
    xs = x.cpu().numpy()
    true = float(np.linalg.norm(system.b - Asp @ xs) / np.linalg.norm(system.b))
    log(f"learned {cfg}: {t:.4f} s/solve iters={d['iters']} resid={true:.3e}")
    return {"s": t, "config": {"restart": cfg[0], "inner_cap": cfg[0] * cfg[1], "poly_degree": cfg[2]},
            "iters": d["iters"], "status": B.status_string(st), "rel_resid_true": true,
            "converged": bool(true <= 1e-10), "sol_err_vs_u": rel_err(xs, system.u),
            "includes": "features + network + polynomial set-up + solve", "x": xs}


def extras(args, ws, learned=True):
    """One timed solve each (after a warm-up) on the 2D 1000^2 and 3D 150^3
    systems: GMRES-IR fp32 and fp64 GMRES (150^3 also with a degree-10
    polynomial, set-up excluded) and the learned-parameter variant.
    The oracle's whole solves of these systems take minutes, so each result
    carries its error against the manufactured u and against the fp64 GMRES
    solution instead, and sol_err_vs_oracle is null with the reason."""
    import numpy as np
    import torch

    from paper_2109_01232_amd import binding as B
    from paper_2109_01232_amd import problems as P

    res = {}
    for key, make, m, cases in (
            ("convdiff2d_1000^2_5pt_seed0", lambda: P.convdiff2d_system(0), 50,
             [("fp32", "fp32", 0), ("fp64", "fp64", 0)]),
            ("aniso3d_150^3_7pt_seed0", lambda: P.aniso3d_system(0), 100,
             [("fp32", "fp32", 0), ("fp32", "fp32", 10), ("fp64", "fp64", 0)])):
        log("extra", key)
        s = make()
        Mx = B.Matrix.from_csr(s.A)
        bx = torch.from_numpy(s.b).cuda()
        xx = torch.zeros_like(bx)
        Asp = s.A.scipy()
        rows, xsol = {}, {}
        for inner, basis, deg in cases:
            roots = B.gmresir_poly_setup(Mx, deg, seed=12345, ws=ws) if deg else None
            p = B.make_params(restart=m, inner=inner, basis=basis, rtol=1e-10, check_mode=1, poly_degree=deg)
            xx.zero_()
            B.gmresir_solve(Mx, bx, xx, p, poly_roots=roots, ws=ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xx.zero_()
            st, d, _ = B.gmresir_solve(Mx, bx, xx, p, poly_roots=roots, ws=ws)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            xs = xx.cpu().numpy()
            true = float(np.linalg.norm(s.b - Asp @ xs) / np.linalg.norm(s.b))
            label = f"{inner}" + (f"_poly{deg}" if deg else "")
            rows[label] = {"s": t, "iters": d["iters"], "status": B.status_string(st), "rel_resid_true": true,
                           "converged": bool(true <= 1e-10), "sol_err_vs_u": rel_err(xs, s.u),
                           "sol_err_vs_oracle": None}
            xsol[label] = xs
            log(f"  {label}: {t:.4f} s iters={d['iters']} resid={true:.2e}")
        if learned and os.path.exists(
                os.path.join(ROOT, "paper_2109_01232_amd", "chooser_weights.json")):
            lv = learned_variant(Mx, bx, xx, ws, s, Asp, 1)
            xsol["learned"] = lv.pop("x")
            lv["sol_err_vs_oracle"] = None
            rows["learned"] = lv
        if "fp64" in rows:
            for k, v in rows.items():
                v["speedup_vs_fp64"] = rows["fp64"]["s"] / v["s"]
                if k in xsol and k != "fp64":
                    v["sol_err_vs_fp64_gmres"] = rel_err(xsol[k], xsol["fp64"])
        res[key] = {"N": s.A.n, "nnz": s.A.nnz, "restart": m, "solves": rows,
                    "oracle": "not run in the default line: the CPU oracle's whole solve of this system takes "
                              "minutes; errors against the manufactured u and the fp64 GMRES solution instead"}
        Mx.close()
        del Mx
    return res


def spmv_study(calls=1000, reps=3):
    """fp64 vs fp32 SpMV time over constant-coefficient stencil families
    (2D on 1500^2, 3D on 130^3 grids), beside the paper's cache model
    5w / (2w + 1) (perfect reuse of x in fp32, none in fp64)."""
    import numpy as np
    import torch

    from paper_2109_01232_amd import binding as B
    from paper_2109_01232_amd import problems as P

    for name in P.STENCILS:
        dim = P.STENCILS[name][0]
        n = 1500 if dim == 2 else 130
        A = P.stencil_matrix(name, n)
        M = B.Matrix.from_csr(A)
        x = np.random.default_rng(0).uniform(-1, 1, A.n)
        rec = {"metric": "spmv_study", "stencil": name, "N": A.n, "nnz": A.nnz,
               "nnz_per_row": A.nnz / A.n, "max_row_nnz": int(np.diff(A.rowptr).max()), "layout": M.layout}
        for prec, dt, sv in (("fp64", torch.float64, 8), ("fp32", torch.float32, 4)):
            xd = torch.from_numpy(x).to(dt).cuda()
            yd = torch.empty_like(xd)
            for _ in range(10):
                B.gmresir_spmv(M, xd, yd, prec)
            best = float("inf")
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(calls):
                    B.gmresir_spmv(M, xd, yd, prec)
                e1.record()
                torch.cuda.synchronize()
                best = min(best, e0.elapsed_time(e1) * 1e3 / calls)
            alg = (sv + 4) * A.nnz + 4 * (A.n + 1) + 2 * sv * A.n
            rec[prec + "_us"] = best
            rec[prec + "_GBps_csr_bytes"] = alg / (best * 1e-6) / 1e9
        w = A.nnz / A.n
        rec["speedup_fp32"] = rec["fp64_us"] / rec["fp32_us"]
        rec["model_speedup"] = 5 * w / (2 * w + 1)
        log(f"spmv {name}: fp64 {rec['fp64_us']:.1f} us, fp32 {rec['fp32_us']:.1f} us, "
            f"x{rec['speedup_fp32']:.2f} (model {rec['model_speedup']:.2f})")
        print(json.dumps(rec), flush=True)
        M.close()
        del M


def time_solves(M, b, p, roots, ws, steps):
    import torch

    from paper_2109_01232_amd import binding as B

    x = torch.zeros_like(b)
    x.zero_()
    B.gmresir_solve(M, b, x, p, poly_roots=roots, ws=ws)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        st, d, _ = B.gmresir_solve(M, b, x, p, poly_roots=roots, ws=ws)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, st, d, x


def suite(args):
    """Time-to-1e-10 on the other configurations and variants (one JSON line
    per solve).  A case is (inner, basis, restart, degree, extra) with extra
    one of {}, {"bj": block size}, {"fd": switch point} or {"poly_prec": "fp32"}
    (an fp32 polynomial applied to fp64 vectors in fp64 GMRES)."""
    import numpy as np
    import torch

    from paper_2109_01232_amd import binding as B
    from paper_2109_01232_amd import problems as P

    steps = max(1, min(args.steps, 3))
    ws = B.Workspace()

    def laplace3d(n):
        # stand-in for the paper's Laplace3D200 (Galeri 7-point Laplacian on a
        # 200^3 grid): b = ones, the paper's default right-hand side
        A = P.stencil_matrix("laplace3d_7", n)
        return P.System(f"laplace3d_{n}", A, np.ones(A.n), None, dict(n=n, rhs="ones"))

    c = lambda inner, basis, m, deg=0, **extra: (inner, basis, m, deg, extra)
    # systems are generated only for the cases that run
    cases = [
        ("aniso3d_150_7pt", lambda: P.aniso3d_system(0),
         [c("fp64", "fp64", 100), c("fp32", "fp32", 100), c("fp32", "fp32", 100, ortho="dcgs2"),
          c("fp32", "fp32", 100, 10), c("fp32", "fp32", 100, 10, ortho="dcgs2"), c("fp32", "fp32", 100, 20),
          c("fp32", "fp32", 100, 30), c("fp32", "fp32", 100, 40),
          c("fp64", "fp64", 100, 10), c("fp64", "fp64", 100, 10, poly_prec="fp32"),
          c("fp64", "fp64", 100, 40), c("fp64", "fp64", 100, 40, poly_prec="fp32")]),
        ("varcoef27_128", lambda: P.varcoef27_system(0),
         [c("fp64", "fp64", 50), c("fp32", "fp32", 50), c("fp32", "bf16", 50), c("fp32", "fp32", 50, ortho="dcgs2"),
          c("fp64", "fp64", 50, ortho="dcgs2")]),
        # GMRES-FD switch points and block Jacobi on the 2D system (Sections "GMRES-IR vs GMRES-FD",
        # "SpMV Speedup: A Large Test Set")
        ("convdiff2d_1000", lambda: P.convdiff2d_system(0),
         [c("fp64", "fp64", 50), c("fp32", "fp32", 50), c("fp32", "fp32", 50, ortho="dcgs2"),
          c("fp64", "fp64", 50, ortho="dcgs2")]
         + [c("fp32", "fp32", 50, fd=sw) for sw in (500, 1000, 2000)]
         + [c("fp32", "fp32", 50, bj=bs) for bs in (8, 16, 32, 42, 64)]),
        # the paper's two 3D Laplacian studies: the IR-vs-FD switch point (Section "GMRES-IR vs
        # GMRES-FD") and the fp32 polynomial's loss of accuracy over degrees 10..70 in fp64 GMRES
        # (Section "Convergence and Kernel Speedup for Preconditioned GMRES vs GMRES-IR")
        ("laplace3d_200", lambda: laplace3d(200),
         [c("fp64", "fp64", 50), c("fp32", "fp32", 50)]
         + [c("fp32", "fp32", 50, fd=sw) for sw in (250, 500, 1000, 2000, 3000)]
         + [c("fp64", "fp64", 50, d, **pp) for d in (10, 20, 30, 40, 50, 60, 70)
            for pp in ({}, {"poly_prec": "fp32"})]),
    ]
    for seed in range(1, 5):
        # the 2D system at its other seeds (Peclet number drawn per seed)
        cases.append((f"convdiff2d_1000_seed{seed}", lambda seed=seed: P.convdiff2d_system(seed),
                      [c("fp64", "fp64", 50), c("fp32", "fp32", 50)]))
    for seed in (1, 2):
        # the 3D systems at their other seeds (the 27-point coefficients and u, or u alone, per seed)
        cases.append((f"varcoef27_128_seed{seed}", lambda seed=seed: P.varcoef27_system(seed),
                      [c("fp64", "fp64", 50), c("fp32", "fp32", 50), c("fp32", "bf16", 50)]))
        cases.append((f"aniso3d_150_7pt_seed{seed}", lambda seed=seed: P.aniso3d_system(seed),
                      [c("fp64", "fp64", 100), c("fp32", "fp32", 100), c("fp32", "fp32", 100, 10)]))
    cases.append(("convdiff2d_64_parity", P.parity_system,
                  [c("fp64", "fp64", 50), c("fp32", "fp32", 50), c("fp32", "bf16", 50)]))

    def label_of(name, inner, basis, m, deg, extra):
        tail = "".join(f"/{k}{v}" for k, v in sorted(extra.items()))
        return f"{name}/{inner}/{basis}/{m}/{deg}{tail}"

    for name, make_system, cfgs in cases:
        labels = [label_of(name, *cf) for cf in cfgs]
        if args.suite_case and not any(args.suite_case in lb for lb in labels):
            continue
        log("suite", name)
        sysm = make_system()
        # set-up of the matrix (CSR upload, fp32 copy, sliced copy): timed, reported, not in the solve times
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M = B.Matrix.from_csr(sysm.A)
        torch.cuda.synchronize()
        t_matrix = time.perf_counter() - t0
        b = torch.from_numpy(np.asarray(sysm.b, dtype=np.float64)).cuda()
        Asp = sysm.A.scipy()
        bnorm = float(np.linalg.norm(sysm.b))
        for (inner, basis, m, deg, extra), label in zip(cfgs, labels):
            if args.suite_case and args.suite_case not in label:
                continue
            roots, t_setup = None, 0.0
            if deg > 0:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                roots = B.gmresir_poly_setup(M, deg, seed=12345, ws=ws)
                torch.cuda.synchronize()
                t_setup = time.perf_counter() - t0
            kw = dict(restart=m, inner=inner, basis=basis, rtol=1e-10, check_mode=1, poly_degree=deg,
                      poly_prec=extra.get("poly_prec"), bj_block=extra.get("bj", 0), ortho=extra.get("ortho", 0),
                      max_iters=args.max_iters)
            p = B.make_params(**kw)
            if "fd" in extra:
                x = torch.zeros_like(b)
                B.gmresir_solve_fd(M, b, x, p, extra["fd"], ws=ws)  # warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    x.zero_()
                    st, d, _ = B.gmresir_solve_fd(M, b, x, p, extra["fd"], ws=ws)
                torch.cuda.synchronize()
                t = (time.perf_counter() - t0) / steps
                gbps = {}
            else:
                t, st, d, x = time_solves(M, b, p, roots, ws, steps)
                x.zero_()
                _, dp, _ = B.gmresir_solve(M, b, x, B.make_params(profile=1, **kw), poly_roots=roots, ws=ws)
                gbps = {k: (dp["cat_bytes"][k] / dp["cat_time_s"][k] / 1e9) for k in B.CATEGORIES
                        if dp["cat_time_s"][k] > 0}
                x.zero_()
                B.gmresir_solve(M, b, x, p, poly_roots=roots, ws=ws)
            xs = x.cpu().numpy()
            true = float(np.linalg.norm(sysm.b - Asp @ xs) / bnorm)
            rec = {"suite": name, "case": label, "N": sysm.A.n, "nnz": sysm.A.nnz,
                   "meta": {k: v for k, v in sysm.meta.items() if isinstance(v, (int, float, str))},
                   "inner": inner, "basis": basis, "restart": m, "poly_degree": deg, **extra,
                   "status": B.status_string(st), "time_to_1e-10_s": t, "poly_setup_s": t_setup,
                   "matrix_setup_s": t_matrix, "layout": M.layout,
                   "iters": d["iters"], "refinements": d["refinements"], "rel_resid_true": true,
                   "converged": bool(true <= 1e-10),
                   "sol_err_vs_u": (rel_err(xs, sysm.u) if sysm.u is not None else None),
                   "GBps_by_category": gbps}
            log(f"  {label}: {t:.4f} s iters={d['iters']} restarts={d['refinements']} resid={true:.2e}")
            print(json.dumps(rec), flush=True)
        M.close()
        del M


if __name__ == "__main__":
    main()
