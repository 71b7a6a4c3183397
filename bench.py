"""Benchmark: eigenpairs/s of the shift-and-invert Jacobi-Davidson solve on one MI355X.

One step = one complete solve (every hot-path step: stencil products, multilevel
preconditioner applies, projected simplified QMR, Gram-Schmidt, Rayleigh-Ritz,
acceptance) of the 10 eigenpairs nearest 0 of the Anderson matrix on the periodic
100^3 lattice, W = 16.5, seed 0, binary32 inner / binary64 outer, tol 1e-10.
The setup (matching, multilevel factorisation, upload) runs once before the timed
region and is reported separately, as is the same solve in plain binary64.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, default=100)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seeds", type=str, default="",
                    help="comma-separated extra disorder seeds: one setup and one solve each, reported as 'seeds'")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=16, help="0 disables the serving leg")
    ap.add_argument("--serve-workers", type=int, default=8)
    ap.add_argument("--serve-warmup", type=int, default=8,
                    help="closed-loop requests that measure the saturated rate before the Poisson stream")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="Poisson arrival rate in req/s (0: 0.8 of the warm-up's saturated rate)")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the serving stream (for long streams such as the 256-request mix)")
    ap.add_argument("--sweep", action="store_true",
                    help="preconditioner parameter study (kappa, epsilon, z_drop, last-level size, segments) "
                         "at the benchmark lattice: one JSON line per setting")
    ap.add_argument("--table5", action="store_true",
                    help="the epsilon x kappa grid of the paper's Table 5 (use with --L 70 --k 5): one JSON "
                         "line per setting")
    ap.add_argument("--lanczos", action="store_true",
                    help="JD against shift-and-invert Lanczos on one setup of the benchmark lattice "
                         "(binary64 and binary32-factor splits): one JSON line")
    ap.add_argument("--kernels-only", action="store_true",
                    help="setup, then only launches of the dominant kernel and a 256 MB copy "
                         "(for hardware counter runs)")
    return ap.parse_args()


def kernels_only(jd, torch, L, reps=20):
    """Launches for counter collection: the binary32 segment products (one apply to fill
    the workspace, then the products of both directions alternately) and, as the
    calibration reference, a plain 256 MB device copy."""
    print("# kernels-only: setup", file=sys.stderr, flush=True)
    prob = jd.Problem(L, 16.5, 0, 0.0, precision="mixed")
    print("# kernels-only: setup done", file=sys.stderr, flush=True)
    pc = prob.precond()
    n = L ** 3
    s = torch.cuda.current_stream()
    x = torch.randn(n, dtype=torch.float32, device="cuda")
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    pc.apply(x, y, "mixed", stream=s)
    for r in range(reps):
        pc.factor_product(None, None, transpose=r % 2, stream=s)
    a = torch.ones(64 * 2 ** 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"kernels_only": True, "nnz": pc.factor_nnz(), "n": n, "reps": reps,
                      "segments": pc.segments(), "copy_bytes_each_way": a.numel() * 4}), flush=True)
    pc.close()
    prob.close()


def stencil_bandwidth(jd, torch, L, W, seed, reps=50):
    """Achieved bandwidth of the binary32 stencil product (secondary kernel), timed with
    events on its stream; algorithmic bytes 3 n 4 (x and eps read, y written)."""
    n = L ** 3
    s = torch.cuda.current_stream()
    eps64 = torch.empty(n, dtype=torch.float64, device="cuda")
    eps32 = torch.empty(n, dtype=torch.float32, device="cuda")
    jd.gen_diag(L, W, seed, eps64, eps32, stream=s)
    # rotate buffers so the 256 MB last-level cache cannot hold the working set
    nbuf = max(2, int(2 * 512e6 / (8 * n)) + 1)
    xs = [torch.randn(n, dtype=torch.float32, device="cuda") for _ in range(nbuf)]
    ys = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(nbuf)]
    for i in range(nbuf):
        jd.stencil_spmv(L, eps32, 0.0, xs[i], ys[i], "mixed", stream=s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for r in range(reps):
        jd.stencil_spmv(L, eps32, 0.0, xs[r % nbuf], ys[r % nbuf], "mixed", stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    b = 3 * n * 4
    return {"kernel": "k_stencil<float>", "bytes_per_launch": b, "avg_us": round(us, 2),
            "achieved_GBs": round(b / (us * 1e-6) / 1e9, 1)}


def block_products(jd, torch, n, reps=10):
    """The Rayleigh-Ritz block products V S on the FP64 matrix cores at the benchmark's
    sizes: the restart (60 -> 20 columns) and a deflation (60 -> 59).  Bytes: V read
    once and the output written (8 n (m + mout)); flops 2 n m mout; HIP events."""
    s = torch.cuda.current_stream()
    out = []
    for m, mout in ((60, 20), (60, 59)):
        V = torch.randn(m, n, dtype=torch.float64, device="cuda").t()
        S = torch.randn(mout, m, dtype=torch.float64, device="cuda").t()
        O = torch.empty(mout, n, dtype=torch.float64, device="cuda").t()
        jd.block_product(V, S, O, stream=s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            jd.block_product(V, S, O, stream=s)
        e1.record(s)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        b, f = 8 * n * (m + mout), 2 * n * m * mout
        out.append({"kernel": "k_gemm_vs", "m": m, "mout": mout, "avg_us": round(us, 1),
                    "GBs": round(b / (us * 1e-6) / 1e9, 1), "TFLOPs": round(f / (us * 1e-6) / 1e12, 2),
                    "hbm_frac": round(b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 3),
                    "mfma_frac": round(f / (us * 1e-6) / 1e12 / 78.6, 3)})
        del V, S, O
    return out


def product_bytes(pc, n, sv=4, sx=4):
    """Algorithmic bytes of the 2 S segment products of one apply (the CSR definition of
    each product, not the layout: entries (value + 4-byte index), row pointers (8 bytes),
    each input element read once, each output element written once, and the output
    permutation of the last product).  Down product s: the r_s unknowns entering the
    segment's first level are its rows and its inputs.  Up product s >= 1: its u_s pivots
    are the rows, its entries those of Z_s less the r_s - u_s unit diagonals of the
    other rows; up product 0: every unknown."""
    seg = pc.segments()
    lv = pc.levels()
    piv = []
    for i, a in enumerate(seg["lev_begin"]):
        b = seg["lev_begin"][i + 1] if i + 1 < seg["segments"] else lv["levels"]
        piv.append(sum(lv["nB"][a:b]))
    total = 0
    for i in range(seg["segments"]):
        r, z = seg["rows"][i], seg["nnz"][i]
        total += z * (sv + 4) + (r + 1) * 8 + 2 * r * sx                      # down
        if i == 0:
            total += z * (sv + 4) + (n + 1) * 8 + 2 * n * sx + 4 * n         # up, all rows
        else:
            u = piv[i]
            total += (z - (r - u)) * (sv + 4) + (u + 1) * 8 + (r + u) * sx  # up, pivots
    return total, 2 * seg["segments"], seg


def factor_roofline(torch, prob, n, reps=40):
    """Roofline of the dominant kernel, the binary32 products with the segments of the
    inverse factor (k_hyb_spmv<float, float>, 2 S launches per preconditioner apply).
    Timed with events on the launch stream over `reps` alternating down / up passes of the
    timing form (the products alone, on the values one apply left in the workspace);
    achieved = the passes' algorithmic bytes / their time, i.e. per launch the mean bytes
    over the mean duration."""
    pc = prob.precond()
    s = torch.cuda.current_stream()
    x = torch.randn(n, dtype=torch.float32, device="cuda")
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    pc.apply(x, y, "mixed", stream=s)
    for t in (0, 1):
        pc.factor_product(None, None, transpose=t, stream=s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for r in range(reps):
        pc.factor_product(None, None, transpose=r % 2, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    pair_bytes, launches, seg = product_bytes(pc, n)
    us_pair = e0.elapsed_time(e1) * 1e3 / (reps / 2)
    b = pair_bytes / launches
    us = us_pair / launches
    achieved = b / (us * 1e-6) / 1e9
    out = {"kernel": "k_hyb_spmv<float, float>", "bound": "hbm", "achieved": round(achieved, 1),
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
           "bytes_per_launch": int(b), "avg_us": round(us, 2), "launches_per_apply": launches,
           "nnz": int(pc.factor_nnz()), "segments": seg, "reps": reps}
    pc.close()
    return out


def apply_roofline(torch, prob, n, reps=20):
    """The whole preconditioner apply (binary32), timed with events on its stream, against
    two byte counts: the bytes the segmented products and the other kernels of the apply
    must move, and the bytes of the multilevel factorisation the apply stands for (each
    level's coupling block L21 traversed twice, down and up: nnz(G) (4 value + 4 index)
    plus the level's rows; block diagonal; the dense last level; input and output)."""
    pc = prob.precond()
    lv = pc.levels()
    s = torch.cuda.current_stream()
    x = torch.randn(n, dtype=torch.float32, device="cuda")
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    for _ in range(3):
        pc.apply(x, y, "mixed", stream=s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        pc.apply(x, y, "mixed", stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    nc = lv["sizes"][-1]
    ld = (nc + 63) // 64 * 64
    prod, launches, _ = product_bytes(pc, n)
    other = 3 * n * 4 + 4 * n + (3 * 4 + 4) * n + 2 * n * 4 + nc * ld * 4 + 3 * nc * 4  # gather, D^-1, last level
    impl = prod + other
    nnz_g = sum(lv["nnzG"])
    method = 2 * nnz_g * 8 + 2 * sum(lv["sizes"][:-1]) * 4 + 2 * n * 4 + nc * nc * 4 + 2 * n * 4 + 2 * n * 4
    pc.close()
    # + the input gather, D^-1 with the last level's gather, and the last level's product
    return {"avg_us": round(us, 1), "launches": launches + 3, "bytes": int(impl),
            "achieved_GBs": round(impl / (us * 1e-6) / 1e9, 1), "frac": round(impl / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "method_bytes": int(method), "nnz_G": int(nnz_g),
            "method_GBs": round(method / (us * 1e-6) / 1e9, 1),
            "method_frac": round(method / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}


SWEEP = [dict()] + [dict(kappa=v) for v in (2.5, 10.0, 20.0)] + [dict(drop_tol=v) for v in (1e-2, 5e-3, 2.5e-3)] \
    + [dict(z_drop=v) for v in (2e-2, 5e-3)] + [dict(coarse_max=v) for v in (4096, 8192)] \
    + [dict(z_parts=v) for v in (1, 4, 8)]
# the grid of the paper's Table 5 (epsilon x kappa, at M = 70, five eigenvalues nearest 0)
TABLE5 = [dict(drop_tol=e, kappa=k) for k in (5.0, 10.0, 20.0) for e in (1e-2, 5e-3, 2.5e-3, 1e-3)]


def sweep(jd, torch, L, k, tol=1e-10, settings=None):
    """Table 5 of the paper, on the GPU: the multilevel preconditioner's parameters one at
    a time around the defaults (kappa 5, epsilon 1/sqrt(n), z_drop min(1e-2, 10 epsilon),
    last level <= 1536, 6 segments): setup time, levels, fill, nnz of the coupling blocks
    and of the inverse factor's segments, the binary32 apply, and the solves."""
    import numpy as np
    n = L ** 3
    rows = []
    for cfg in settings if settings is not None else SWEEP:
        t0 = time.time()
        prob = jd.Problem(L, 16.5, 0, 0.0, precision="mixed", **cfg)
        setup = time.time() - t0
        pc = prob.precond()
        lv, seg = pc.levels(), pc.segments()
        s = torch.cuda.current_stream()
        x = torch.randn(n, dtype=torch.float32, device="cuda")
        y = torch.empty(n, dtype=torch.float32, device="cuda")
        for _ in range(3):
            pc.apply(x, y, "mixed", stream=s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(10):
            pc.apply(x, y, "mixed", stream=s)
        e1.record(s)
        torch.cuda.synchronize()
        info = prob.info()
        row = {"setting": cfg or "defaults", "setup_s": round(setup, 2), "levels": info["levels"],
               "coarse_n": info["coarse_n"], "fill": round(info["fill"], 3), "nnz_G": int(sum(lv["nnzG"])),
               "nnz_Z": int(pc.factor_nnz()), "segments": seg["segments"], "device_bytes": int(info["device_bytes"]),
               "apply_us": round(e0.elapsed_time(e1) * 100, 1)}
        pc.close()
        for prec in ("mixed", "fp64"):
            prob.set_precision(prec)
            ev, _, res, i2 = prob.solve(k, tol)
            row[prec] = {"solve_s": round(i2["solve_s"], 3), "outer": i2["outer_its"], "inner": i2["inner_its"],
                         "converged": i2["n_converged"], "max_resid": float(np.nanmax(res))}
        prob.close()
        print(json.dumps(row), flush=True)
        rows.append(row)
    return rows


def lanczos_leg(jd, L, k, tol=1e-10, W=16.5, seed=0, sigma=0.0):
    """Section 4.1 / Tables 2-3 of the paper on the GPU: the same k pairs nearest sigma by
    Jacobi-Davidson and by shift-and-invert Lanczos (each product with (A - sigma I)^-1 an
    SQMR solve to 1e-10 with the same multilevel preconditioner), from one setup, with
    binary64 vectors and binary64 or binary32 factors."""
    import numpy as np
    t0 = time.time()
    prob = jd.Problem(L, W, seed, sigma, precision="mixed")
    setup = time.time() - t0
    print(f"# lanczos leg: setup {setup:.1f} s", file=sys.stderr, flush=True)
    out = {"L": L, "W": W, "seed": seed, "sigma": sigma, "k": k, "tol": tol, "setup_s": round(setup, 2)}
    for prec in ("fp64", "mixed_factors"):
        prob.set_precision(prec)
        ev_jd, _, res_jd, i_jd = prob.solve(k, tol)
        print(f"# {prec} JD {i_jd['solve_s']:.3f} s", file=sys.stderr, flush=True)
        ev_l, _, res_l, i_l = prob.lanczos(k, tol)
        print(f"# {prec} SI-Lanczos {i_l['solve_s']:.3f} s", file=sys.stderr, flush=True)
        out[prec] = {
            "jd": {"solve_s": round(i_jd["solve_s"], 3), "outer": i_jd["outer_its"], "inner": i_jd["inner_its"],
                   "converged": i_jd["n_converged"], "max_resid": float(np.nanmax(res_jd))},
            "si_lanczos": {"solve_s": round(i_l["solve_s"], 3), "products": i_l["outer_its"], "inner": i_l["inner_its"],
                           "converged": i_l["n_converged"], "status": i_l["status"],
                           "max_resid": float(np.nanmax(res_l))},
            "max_abs_eval_diff": float(np.nanmax(np.abs(np.sort(ev_jd) - np.sort(ev_l)))),
        }
    prob.close()
    return out


def serving(jd, nreq, workers, warm=8, rate=None):
    """The server on the mixed request stream: a closed-loop warm-up measures the
    saturated request rate, then nreq requests arrive as a Poisson process at 0.8 of
    that rate (or at `rate` req/s when given); latency = submission -> completion
    (measured by the server)."""
    import numpy as np
    from tests import seeded_inputs
    reqs = seeded_inputs.serving_requests(warm + nreq)
    mk = lambda r: jd.Server.request(r["L"], r["W"], r["seed"], r["sigma"], r["k"], 1e-10, "mixed")
    srv = jd.Server(workers=workers)

    def run(batch, arrivals, label):
        # submit each request at its arrival time and report every completion
        t0, i, pending, res = time.time(), 0, {}, [None] * len(batch)
        while i < len(batch) or pending:
            now = time.time() - t0
            while i < len(batch) and (arrivals is None or arrivals[i] <= now):
                pending[srv.submit(mk(batch[i]))] = i
                i += 1
            for t, j in list(pending.items()):
                r = srv.poll(t)
                if r is None:
                    continue
                res[j] = r
                del pending[t]
                q = batch[j]
                print(f"# serving {label} {j}: L={q['L']} W={q['W']} k={q['k']} status {r['status']} "
                      f"setup {r['setup_s']:.2f} s solve {r['solve_s']:.2f} s latency {r['latency_s']:.2f} s",
                      file=sys.stderr, flush=True)
            time.sleep(0.01)
        return res, time.time() - t0

    _, span = run(reqs[:warm], None, "warm-up")
    sat = warm / span
    lam = rate if rate else 0.8 * sat
    print(f"# serving: saturated {sat:.2f} req/s, Poisson arrivals at {lam:.2f} req/s", file=sys.stderr, flush=True)
    res, span = run(reqs[warm:], seeded_inputs.poisson_arrivals(nreq, lam), "poisson")
    srv.close()
    for r, q in zip(res, reqs[warm:]):
        if r["status"] != 0:
            print(f"# serving: request {q} -> status {r['status']}, {r['n_converged']}/{r['k']} converged, "
                  f"outer {r['outer_its']}, {r['error']}", file=sys.stderr, flush=True)
    lat = np.array([r["latency_s"] for r in res])
    ok = sum(r["status"] == 0 for r in res)
    pairs = sum(r["n_converged"] for r in res)
    return {"requests": nreq, "workers": workers, "setup_threads": "adaptive",
            "saturated_rps": round(sat, 3), "arrival_rps": round(lam, 3),
            "completed_ok": int(ok), "p50_latency_s": round(float(np.percentile(lat, 50)), 3),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 3),
            "p50_setup_s": round(float(np.percentile([r["setup_s"] for r in res], 50)), 3),
            "p50_solve_s": round(float(np.percentile([r["solve_s"] for r in res], 50)), 3),
            "p99_solve_s": round(float(np.percentile([r["solve_s"] for r in res], 99)), 3),
            "p50_queued_s": round(float(np.percentile([r["queued_s"] for r in res], 50)), 3),
            "p99_setup_s": round(float(np.percentile([r["setup_s"] for r in res], 99)), 3),
            "p99_queued_s": round(float(np.percentile([r["queued_s"] for r in res], 99)), 3),
            "eigenpairs_per_s": round(pairs / span, 3),
            # where the time goes: host setups against device solves over the stream's
            # wall time (solves of different requests overlap on the GPU)
            "wall_s": round(span, 2), "sum_setup_s": round(sum(r["setup_s"] for r in res), 2),
            "sum_solve_s": round(sum(r["solve_s"] for r in res), 2),
            "workload": "L in {20..60}, W in {12, 16.5, 21}, sigma ~ U[-1,1], k in 1..10, seeds 1e6+i, "
                        "FP32 inner / FP64 outer, tol 1e-10"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(k, L_bench):
    """The oracle (exact multifrontal LDL^T + shift-and-invert Lanczos, binary64) timed
    live on bounded samples, and the stored oracle run of the benchmarked workload.

    Live: the 30^3 lattice with all the box's threads, and again on one thread (the
    paper timed one core).  The 100^3 oracle run takes about 20 minutes on
    8 cores, far beyond the benchmark's budget: its time is quoted from the stored
    result that make_golden.py wrote (its own machine, stated there)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import eig, generator
    W, seed, sigma = 16.5, 0, 0.0
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    threads = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    L = 30
    eps = generator.disorder(L, W, seed)
    t0 = time.time()
    lams, X, res, anorm = eig.nearest_eigenpairs(L, eps, sigma, k)
    dt = time.time() - t0
    L1 = 30
    eps1 = eps
    with threadpool_limits(limits=1):
        t1 = time.time()
        eig.nearest_eigenpairs(L1, eps1, sigma, k)
        dt1 = time.time() - t1
    out = {"value": round(k / dt, 4), "unit": "eigenpairs/s", "cores": threads, "kind": "oracle",
           "cpu_model": _cpu_model(),
           "sample": f"L={L} (n={L**3}), W={W}, seed {seed}, sigma 0, k={k}: exact LDL^T + SI-Lanczos, "
                     f"{dt:.1f} s on {threads} threads",
           "max_residual_over_anorm": float(np.max(res) / anorm),
           "one_core": {"value": round(k / dt1, 4), "unit": "eigenpairs/s", "cores": 1,
                        "sample": f"L={L1} (n={L1**3}), same parameters, {dt1:.1f} s on one thread"}}
    gold = os.path.join(ROOT, "tests", "golden", f"L{L_bench}_W16.5_s0_k{k}.json")
    if os.path.exists(gold):
        with open(gold) as fh:
            g = json.load(fh)
        cert = g.get("certificate", {})
        out["stored_full_size"] = {
            "workload": f"L={L_bench}, W=16.5, seed 0, sigma 0, k={k} (the benchmarked workload)",
            "reference": os.path.relpath(gold, ROOT), "seconds": g.get("seconds"),
            "value": round(k / g["seconds"], 5) if g.get("seconds") else None, "unit": "eigenpairs/s",
            "factorisation_s": g.get("factor_seconds"), "lanczos_s": g.get("lanczos_seconds"),
            "machine": g.get("machine", "the build container (8 threads, Intel Xeon @ 2.70GHz)"),
            "inertia_certificate_s": cert.get("seconds")}
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not implemented)"}))
        sys.exit(2)
    import numpy as np
    import torch
    import paper_math_0508111_amd as jd

    torch.cuda.set_device(0)
    if a.kernels_only:
        kernels_only(jd, torch, a.L)
        return
    if a.sweep or a.table5:
        rows = sweep(jd, torch, a.L, a.k, settings=TABLE5 if a.table5 else None)
        print(json.dumps({"sweep": rows, "L": a.L, "k": a.k}), flush=True)
        return
    if a.lanczos:
        print(json.dumps({"lanczos": lanczos_leg(jd, a.L, a.k)}), flush=True)
        return
    if a.serve_only:
        print(json.dumps({"serving": serving(jd, a.serve_requests, a.serve_workers, a.serve_warmup, a.serve_rate)}), flush=True)
        return
    L, W, seed, sigma, k, tol = a.L, 16.5, 0, 0.0, a.k, 1e-10
    t0 = time.time()
    prob = jd.Problem(L, W, seed, sigma, precision="mixed")
    setup_wall = time.time() - t0
    pinfo = prob.info()
    print(f"# setup {setup_wall:.2f} s, levels {pinfo['levels']}, coarse {pinfo['coarse_n']}, "
          f"fill {pinfo['fill']:.2f}", file=sys.stderr, flush=True)
    for w in range(a.warmup):
        ev, _, res, info = prob.solve(k, tol)
        print(f"# warmup {w}: {info['solve_s']:.3f} s, outer {info['outer_its']}, inner {info['inner_its']}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.time()
    infos = []
    for step in range(a.steps):
        ev, _, res, info = prob.solve(k, tol)
        infos.append(info)
        print(f"# step {step}: {info['solve_s']:.3f} s, converged {info['n_converged']}, outer {info['outer_its']}, "
              f"inner {info['inner_its']}, max resid {np.nanmax(res):.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.time() - t0
    converged = sum(i["n_converged"] for i in infos)
    value = converged / T
    out = {
        "metric": "eigenpairs/s at L=100,W=16.5 (FP32-inner vs FP64); p50/p99 request latency",
        "value": round(value, 4), "unit": "eigenpairs/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(1e3 * T / a.steps, 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32-inner/f64-outer", "data": "synthetic",
        "config": {"workload": f"Anderson {L}^3 periodic, W=16.5, seed 0, {k} eigenpairs nearest 0, tol 1e-10, "
                               f"FP32 inner / FP64 outer", "L": L, "n": L ** 3, "k": k, "sigma": sigma,
                   "W": W, "tol": tol},
        "setup_s": round(setup_wall, 3), "device_bytes": int(infos[-1]["device_bytes"]),
        "end_to_end": {"value": round(infos[-1]["n_converged"] / (setup_wall + infos[-1]["solve_s"]), 4),
                       "unit": "eigenpairs/s", "what": "one setup (host) plus one solve"},
        "outer_its": infos[-1]["outer_its"], "inner_its": infos[-1]["inner_its"],
        "levels": pinfo["levels"], "coarse_n": pinfo["coarse_n"], "fill": round(pinfo["fill"], 3),
        "max_resid_over_anorm": float(np.nanmax(res)),
        "evals": [float(v) for v in ev],
    }
    if not a.no_fp64:
        # the same setup, other precision splits: binary64 throughout, and binary32
        # preconditioner factors with binary64 vectors
        for name in ("fp64", "mixed_factors"):
            prob.set_precision(name)
            e2, _, r2, i2 = prob.solve(k, tol)
            out[name] = {"value": round(i2["n_converged"] / i2["solve_s"], 4), "solve_s": round(i2["solve_s"], 3),
                         "outer_its": i2["outer_its"], "inner_its": i2["inner_its"],
                         "converged": i2["n_converged"],
                         "max_abs_eval_diff_vs_mixed": float(np.nanmax(np.abs(e2 - ev)))}
            gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                                f"L{L}_W16.5_s{seed}_k{k}.json")
            if os.path.exists(gold):
                with open(gold) as fh:
                    out[name]["oracle_max_abs_err"] = float(np.nanmax(np.abs(e2 - np.array(json.load(fh)["lams"]))))
            print(f"# {name} solve {i2['solve_s']:.3f} s, outer {i2['outer_its']}, inner {i2['inner_its']}",
                  file=sys.stderr, flush=True)
    prob.set_precision("mixed")
    # error of every returned eigenvalue against the stored FP64 oracle result of the same
    # workload (tests/golden, written by a script that calls only the oracle), when there is one
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", f"L{L}_W16.5_s{seed}_k{k}.json")
    if os.path.exists(gold):
        with open(gold) as fh:
            g = json.load(fh)
        if g["sigma"] == sigma and g["k"] == k:
            ref = np.array(g["lams"])
            out["oracle_error"] = {"reference": os.path.relpath(gold, os.path.dirname(os.path.abspath(__file__))),
                                   "method": g["method"], "mixed": [float(v) for v in np.abs(ev - ref)]}
            for name in ("fp64", "mixed_factors"):
                if name in out:
                    out["oracle_error"][name + "_max"] = out[name].get("oracle_max_abs_err")
    out["roofline"] = factor_roofline(torch, prob, L ** 3)
    out["apply"] = apply_roofline(torch, prob, L ** 3)
    out["stencil"] = stencil_bandwidth(jd, torch, L, W, seed)
    out["block_products"] = block_products(jd, torch, L ** 3)
    prob.close()
    if a.seeds:
        # seed-to-seed spread of the same workload (other disorder realisations)
        out["seeds"] = []
        for sd in [int(v) for v in a.seeds.split(",") if v.strip()]:
            p2 = jd.Problem(L, W, sd, sigma, precision="mixed")
            e2, _, r2, i2 = p2.solve(k, tol)
            p2.close()
            out["seeds"].append({"seed": sd, "setup_s": round(i2["setup_s"], 2), "solve_s": round(i2["solve_s"], 3),
                                 "outer_its": i2["outer_its"], "inner_its": i2["inner_its"],
                                 "converged": i2["n_converged"], "value": round(i2["n_converged"] / i2["solve_s"], 4),
                                 "max_resid_over_anorm": float(np.nanmax(r2))})
            print(f"# seed {sd}: setup {i2['setup_s']:.1f} s, solve {i2['solve_s']:.3f} s, outer {i2['outer_its']}, "
                  f"inner {i2['inner_its']}, converged {i2['n_converged']}", file=sys.stderr, flush=True)
    if a.serve_requests > 0:
        out["serving"] = serving(jd, a.serve_requests, a.serve_workers, a.serve_warmup, a.serve_rate)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(k, L)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
