"""Benchmark: sgn(gamma5 Dw(mu)) b solves/s and Wilson-Dirac stencil GB/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

One step is one ovs_sign_apply over a batch of sources resident in HBM:
packing, LR deflation projection (when eigentriples are given), the
two-sided Lanczos loop with per-source convergence checks, the inner sign
sgn(G_k) e_1 and the combination.  The workload (synthetic, seeded):
16^3 x 32 lattice, links P_SU3(1 + 0.6 G), m_w = -1.5, mu = 0.4, 12 Gaussian
sources, FP32 storage with FP64 coefficients, target relative error 1e-5.

Prints one JSON line.  value = solves/s of the timed steps.  The roofline
object is for the dominant kernel of a solve, the dual stencil of the Lanczos
step (A v~ and A^dag w~ with their partial sums), timed on the workload's 12
sources with HIP events on the library stream; `stencil` gives the same for the
plain Wilson stencil A x.
vs_fp64_single_source solves the same sources one at a time on an FP64
lattice (autotuned for one source), without and with graphs, and gives the
batched FP32-storage rate over each.  cpu_baseline times the CPU oracle's
two-sided Lanczos on a bounded sample of the same workload.
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

METRIC = "Dw(μ) stencil GB/s vs HBM peak; sign(A)b solves/s at stated rel. error"
HBM_PEAK_GBS = 8000.0
DIMS = (16, 16, 16, 32)
EPS, MU, MW = 0.6, 0.4, -1.5
NRHS = 12
TOL = 1e-5
KMAX = 1000
SAVED_TUNING = os.path.join(ROOT, "paper_0810_4228_amd", "tuning_mi355x.json")


# HBM bytes per launch of the tuned FP32 kernels on this workload, from the
# FETCH_SIZE / WRITE_SIZE counters scaled by a device copy of known size
# (profiles/*_hbm_counters.txt).  Reported only while the kernel source and
# the autotuner's choice are the ones that were measured.
TRAFFIC = {
    "stencil": {"source_sha256_prefix": "e5fcfd66358a5cde",
                "tuning": {"rhs_block": 1, "wg": 128, "lds_kb": 0, "order": 7, "lanes_per_site": 1, "streaming_store": 1, "staged_tile": 1},
                "bytes_per_launch": 1.9998 * 203985.36 * 1024 + 1.0000 * 147463.60 * 1024},
    "dual": {"source_sha256_prefix": "e5fcfd66358a5cde",
             "tuning": {"rhs_block": 1, "wg": 256, "lds_kb": 53, "order": 4, "variant": "one thread per site", "streaming_store": 1, "update_streaming_store": 1},
             "bytes_per_launch": 1.9998 * 440367.61 * 1024 + 1.0000 * 295164.36 * 1024},
}


def measured_traffic(kind, tuning):
    import hashlib
    t = TRAFFIC[kind]
    if not t["source_sha256_prefix"] or t.get("tuning") != tuning.get(kind):
        return None
    src = os.path.join(ROOT, "paper_0810_4228_amd", "csrc", "stencil.hip")
    try:
        with open(src, "rb") as fh:
            digest = hashlib.sha256(fh.read()).hexdigest()
    except OSError:
        return None
    return t["bytes_per_launch"] if digest.startswith(t["source_sha256_prefix"]) else None


def dual_kernel_name(du):
    """Kernel symbol of the tuned dual-stencil variant (as rocprofv3 lists it)."""
    b = du["rhs_block"]
    return {"one thread per site": f"k_dual<float, {b}>",
            "lane pair": f"k_dual_pair<float, {b}, false>",
            "lane pair, LDS-staged tile": f"k_dual_pair<float, {b}, true>",
            "operator per workgroup": f"k_dual_op<float, {b}, false>",
            "operator per workgroup, LDS-staged tile": f"k_dual_op<float, {b}, true>",
            "operator per workgroup, marching along t": "k_dual_march<float>"}.get(du["variant"], "?")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stencil_bytes(V, nrhs, es):
    """Algorithmic bytes of one A application: links once + input and output fields."""
    return V * (36 * es + 2 * 12 * es * nrhs)


def dual_bytes(V, nrhs, es):
    """Dual Lanczos stencil: links once + read v, w and write A v, A^dag w."""
    return V * (36 * es + 4 * 12 * es * nrhs)


CPU_PROCS = 16   # the host-core share of one GPU on the measurement boxes
CPU_ITERS = 10


def _cpu_worker(r, barrier, out):
    """One oracle process: build the CSR operator of the workload, wait for all
    processes, run CPU_ITERS two-sided Lanczos iterations on source r."""
    import synth
    from oracle import dirac, krylov
    U = synth.random_links(DIMS, EPS, seed=synth.LINK_SEED)
    A = dirac.csr_A(DIMS, U, MW, MU)
    Ad = dirac.csr_A(DIMS, U, MW, -MU)
    del U
    b = synth.gaussian_sources(DIMS, NRHS, seed=synth.SOURCE_SEED)[r % NRHS]
    barrier.wait()
    t0 = time.perf_counter()
    krylov.two_sided_lanczos(lambda v: A @ v, lambda v: Ad @ v, b, b, CPU_ITERS, store=False)
    t = time.perf_counter() - t0
    barrier.wait()
    out.put(t)


def cpu_oracle_timing(procs=CPU_PROCS):
    """Times the oracle's two-sided Lanczos (scipy CSR, FP64) on `procs`
    concurrent single-threaded processes, one source each, CPU_ITERS iterations
    between two barriers.  Runs before this process touches the GPU.  Returns
    (seconds per iteration per process, processes)."""
    import multiprocessing as mp
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                            "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")
        barrier = ctx.Barrier(procs)
        out = ctx.Queue()
        ps = [ctx.Process(target=_cpu_worker, args=(r, barrier, out)) for r in range(procs)]
        for p in ps:
            p.start()
        times = [out.get(timeout=600) for _ in ps]
        for p in ps:
            p.join()
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return float(np.mean(times)) / CPU_ITERS, procs


def cpu_baseline(t_it, procs, k_avg):
    return {
        "value": procs / (t_it * k_avg),
        "unit": "solves/s",
        "cores": procs,
        "kind": "oracle",
        "sample": f"oracle two-sided Lanczos (scipy CSR, FP64), {procs} concurrent single-threaded "
                  f"processes, one of the 12 sources each, {CPU_ITERS} iterations at 16^3x32 "
                  f"({t_it:.3f} s per iteration per process; operator build excluded), scaled to "
                  f"k = {k_avg:.0f} iterations per solve",
    }


def free_field_check(ovs, torch, dev):
    """Same lattice size and code path with unit links: error against the closed form."""
    import synth
    from oracle import freefield
    U = synth.unit_links(DIMS)
    b = synth.gaussian_sources(DIMS, 2, seed=synth.SOURCE_SEED)
    lat = ovs.Lattice(DIMS, precision="f32")
    lat.set_links(torch.from_numpy(U).to(dev))
    lat.set_params(MW, MU)
    y, info, st = lat.sign_apply(torch.from_numpy(b).to(dev), KMAX, tol=TOL, graph=True)
    ref = freefield.free_sign_apply(DIMS, MW, MU, b)
    yc = y.cpu().numpy()
    errs = [float(np.linalg.norm(yc[r] - ref[r]) / np.linalg.norm(ref[r])) for r in range(2)]
    lat.close()
    return max(errs), [i["k_used"] for i in info]


def copy_bandwidth(torch, dev, nbytes=1 << 30, iters=20):
    """Device-to-device copy rate (read + write bytes / time, HIP events): the
    practical HBM ceiling the kernels are also compared with."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / iters
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def overlap_eigs_timing(ovs, torch, dev, dims=(8, 8, 8, 8), nev=4, ncv=80, block=4):
    """ovs_overlap_eigs: the nev eigenvalues of smallest magnitude of D_ov(mu)
    (eps 0.6, mu 0.3, FP64, sign solves to 1e-10, Ritz residuals to 1e-8),
    wall time of one call (its first sign solve allocates the workspace)."""
    import synth
    lat = ovs.Lattice(dims, precision="f64")
    lat.set_links(torch.from_numpy(synth.random_links(dims, 0.6, seed=synth.LINK_SEED)).to(dev))
    lat.set_params(MW, 0.3)
    kw = dict(ncv=ncv, block=block, k_inner=1000, tol_inner=1e-10, tol=1e-8, max_restarts=200)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, _, info, st = lat.overlap_eigs(nev, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
    except Exception as e:  # reported, not fatal to the bench line
        lat.close()
        return {"error": str(e)}
    lat.close()
    return {"workload": "x".join(map(str, dims)) + f", eps 0.6, mu 0.3, FP64, nev {nev}, ncv {ncv}, block {block}",
            "ms": ms, "status": st, "lambda": [[z.real, z.imag] for z in lam], **info,
            "ms_per_sign_solve": ms / max(info["sign_solves"], 1)}


def eig_timing(ovs, torch, dev, dims=(8, 8, 8, 8), eps=0.6, mu=0.3, m=30, tol=1e-10):
    """ovs_deflation_compute: m critical eigentriples (right and left, FP64)
    by shift-invert Krylov-Schur; seconds, status and the solver's info."""
    import synth
    lat = ovs.Lattice(dims, precision="f64")
    lat.set_links(torch.from_numpy(synth.random_links(dims, eps, seed=synth.LINK_SEED)).to(dev))
    lat.set_params(MW, mu)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d, st = lat.deflation_compute(m, tol=tol, max_iter=30)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lam, R, L, info = d.get()
    d.close()
    lat.close()
    return {"workload": "x".join(map(str, dims)) + f", eps {eps}, mu {mu}, m = {m}, tol {tol}",
            "seconds": dt, "status": int(st), "max_rel_residual": float(info[0]),
            "biorth_dev": float(info[1]), "restarts": int(info[2]),
            "abs_lambda_range": [float(abs(lam[0])), float(abs(lam[-1]))]}


def config5(ovs, torch, dev, mu=0.1, m=40, reps=2):
    """The 16^3 x 32 lattice with rough links P_SU3(1 + 0.8 G) at mu = 0.1
    (at mu = 0.4 the method does not converge on these links), 12 Gaussian sources with target tolerances 1e-5 (even) and 1e-8
    (odd), FP32 storage (the 1e-8 group in FP64), LR deflation by m computed
    eigentriples (Sections 3, 5; the deflation phase is timed separately and
    excluded from solves/s, as in the paper), two-pass (one-pass bases for
    k ~ 1350 in both groups would exceed one GPU's memory), graphs.  The
    result is checked by sgn(A)^2 = 1: the same solve applied to y must return
    b.  The same sources without deflation show what it buys."""
    import synth
    dims = DIMS
    lat = ovs.Lattice(dims, precision="f32")
    lat.set_links(torch.from_numpy(synth.random_links(dims, 0.8, seed=synth.LINK_SEED)).to(dev))
    lat.set_params(MW, mu)
    bt = torch.from_numpy(synth.gaussian_sources(dims, NRHS, seed=synth.SOURCE_SEED)).to(dev)
    tol = [1e-5 if j % 2 == 0 else 1e-8 for j in range(NRHS)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d, st_d = lat.deflation_compute(m, tol=1e-10, max_iter=30)
    torch.cuda.synchronize()
    t_defl = time.perf_counter() - t0
    lam, R, L, dinfo = d.get()
    del R, L
    log(f"bench: config 5 eigentriples {t_defl:.1f} s, status {st_d}, info {dinfo}")

    def solve(x, defl):
        # k_max: the deflated solve needs k <= 1350, the undeflated one k <= 3950
        return lat.sign_apply(x, KMAX * 2 if defl is not None else KMAX * 6, defl=defl, tol=tol,
                              graph=True, two_pass=True)
    solve(bt, d)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y, info, st = solve(bt, d)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    y2, _, _ = solve(y.contiguous(), d)
    e2 = (torch.linalg.vector_norm(y2 - bt, dim=1) / torch.linalg.vector_norm(bt, dim=1)).cpu().numpy()
    d.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y0, info0, st0 = solve(bt, None)
    torch.cuda.synchronize()
    dt0 = time.perf_counter() - t0
    lat.close()
    return {"workload": "16x16x16x32, links P_SU3(1+0.8G) seed 0, m_w -1.5, mu 0.1, 12 Gaussian "
                        "sources, tol 1e-5 (even) / 1e-8 (odd), FP32 storage with the 1e-8 group "
                        f"in FP64, {m} computed eigentriples, two-pass, graphs",
            "deflation_phase_s": t_defl, "eigentriples_status": int(st_d),
            "eigentriples_max_rel_residual": float(dinfo[0]), "eigentriples_biorth_dev": float(dinfo[1]),
            "abs_lambda_range": [float(abs(lam[0])), float(abs(lam[-1]))],
            "solves_per_s": NRHS / dt, "ms_per_batch": dt * 1e3, "status": int(st),
            "k_used": [i["k_used"] for i in info], "fp64": [i["fp64"] for i in info],
            "escalated": [i["escalated"] for i in info],
            "est_rel_err_max": max(i["est_rel_err"] for i in info),
            "sign_squared_rel_err": {"tol_1e-5": float(e2[0::2].max()), "tol_1e-8": float(e2[1::2].max())},
            "k_max": KMAX * 2,
            "undeflated": {"solves_per_s": NRHS / dt0, "status": int(st0), "k_max": KMAX * 6,
                           "k_used": [i["k_used"] for i in info0]},
            "mu_0.4": "not converged by k = 6000 with or without the 40 eigentriples (measured; "
                      "not run here)"}


def compare_methods(ovs, torch, dev, dims=(8, 8, 8, 8), mu=0.3, m=30, ks=(200, 400, 600, 800)):
    """The paper's comparison (Section 5, its accuracy-vs-k and accuracy-vs-time
    figures) on the GPU: LR-deflated two-sided Lanczos against LR-deflated
    Arnoldi, FP64, one Gaussian source, eps 0.6, m computed eigentriples, at
    each k: the relative error against the 2sL result at k = 1600 and the
    time of one ovs_sign_apply (no tolerance: exactly k steps; graphs off, as
    Arnoldi has none).  Also times the eigentriples (setup)."""
    import synth
    lat = ovs.Lattice(dims, precision="f64")
    lat.set_links(torch.from_numpy(synth.random_links(dims, 0.6, seed=synth.LINK_SEED)).to(dev))
    lat.set_params(MW, mu)
    b = torch.from_numpy(synth.gaussian_sources(dims, 1, seed=synth.SOURCE_SEED)).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d, st = lat.deflation_compute(m, tol=1e-10, max_iter=30)
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    lam, R, L, info = d.get()
    del R, L
    yref = lat.sign_apply(b, 1600, defl=d)[0].cpu().numpy()[0]
    rows = []
    for k in ks:
        row = {"k": k}
        for meth in ("2sl", "arnoldi"):
            lat.sign_apply(b, k, defl=d, method=meth)  # warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            y = lat.sign_apply(b, k, defl=d, method=meth)[0]
            torch.cuda.synchronize()
            row[meth + "_ms"] = (time.perf_counter() - t1) * 1e3
            yc = y.cpu().numpy()[0]
            row[meth + "_rel_err"] = float(np.linalg.norm(yc - yref) / np.linalg.norm(yref))
        rows.append(row)
    d.close()
    lat.close()
    return {"workload": "x".join(map(str, dims)) + f", eps 0.6, mu {mu}, 1 Gaussian source, FP64, "
                        f"{m} computed eigentriples; reference: 2sL at k = 1600",
            "eigentriples": {"seconds": t_eig, "status": int(st), "max_rel_residual": float(info[0]),
                             "biorth_dev": float(info[1]), "restarts": int(info[2])},
            "rows": rows}


def gradient_timing(ovs, torch, dev, dims=(8, 8, 8, 8), k=400, m_defl=0):
    """ovs_sign_apply_vjp (eps 0.6, mu 0.3, one Gaussian source and cotangent,
    FP64, k iterations) with the Lanczos vectors recomputed from checkpoints and
    with the bases stored, against the k-step forward alone (no tolerance, no
    graphs: the same kernels the sweep uses).  The default is the gradient
    configuration, 8^4 at k = 400.  With m_defl > 0 both run with that many
    computed eigentriples (LR deflation; the eigentriples are computed
    outside the timed region)."""
    import synth
    lat = ovs.Lattice(dims, precision="f64")
    lat.set_links(torch.from_numpy(synth.random_links(dims, 0.6, seed=synth.LINK_SEED)).to(dev))
    lat.set_params(MW, 0.3)
    b = torch.from_numpy(synth.gaussian_sources(dims, 1, seed=synth.SOURCE_SEED)).to(dev)
    chi = torch.from_numpy(synth.gaussian_sources(dims, 1, seed=synth.COTANGENT_SEED)).to(dev)
    d = lat.deflation_compute(m_defl, tol=1e-10, max_iter=30)[0] if m_defl else None

    def t(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    fwd = t(lambda: lat.sign_apply(b, k, defl=d))
    rec = t(lambda: lat.sign_apply_vjp(b, chi, k, defl=d))
    sto = t(lambda: lat.sign_apply_vjp(b, chi, k, store_basis=True, defl=d))
    if d is not None:
        d.close()
    lat.close()
    return {"workload": "x".join(map(str, dims)) + f", eps 0.6, mu 0.3, 1 source, FP64, k = {k}"
                        + (f", {m_defl} deflated eigentriples" if m_defl else ""),
            "forward_ms": fwd, "vjp_recompute_ms": rec, "vjp_stored_basis_ms": sto,
            "ratio_recompute": rec / fwd, "ratio_stored": sto / fwd}


def launch_modes(ovs, torch, dev, lat, bt):
    """Solves/s of captured graphs (the default) against persistent launches:
    the benchmark workload, and 12 sources on an 8^4 lattice (launch-bound)."""
    import synth
    out = {}

    def rate(lt, b, tol, **kw):
        lt.sign_apply(b, KMAX, tol=[tol] * NRHS, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            lt.sign_apply(b, KMAX, tol=[tol] * NRHS, **kw)
        torch.cuda.synchronize()
        return 3 * NRHS / (time.perf_counter() - t0)

    out["16x16x16x32_f32"] = {"graph": rate(lat, bt, TOL, graph=True),
                              "persistent": rate(lat, bt, TOL, persistent=True)}
    dims = (8, 8, 8, 8)
    small = ovs.Lattice(dims, precision="f32")
    small.set_links(torch.from_numpy(synth.random_links(dims, EPS, seed=synth.LINK_SEED)).to(dev))
    small.set_params(MW, MU)
    small.autotune(NRHS)
    bs = torch.from_numpy(synth.gaussian_sources(dims, NRHS, seed=synth.SOURCE_SEED)).to(dev)
    out["8x8x8x8_f32"] = {"graph": rate(small, bs, TOL, graph=True),
                          "persistent": rate(small, bs, TOL, persistent=True)}
    small.close()
    return out


def fp64_single_source(ovs, torch, dev, U, bt, y32, graph, mu=MU):
    """The same sources solved one at a time on an FP64 lattice (same links,
    same tolerance), sequentially: solves/s and the largest relative
    difference from the batched FP32-storage result."""
    lat = ovs.Lattice(DIMS, precision="f64")
    lat.set_links(U)
    lat.set_params(MW, mu)
    lat.autotune(1)
    lat.sign_apply(bt[0:1], KMAX, tol=[TOL], graph=graph)  # warm-up (workspace, graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ys = []
    for r in range(bt.shape[0]):
        y, _, _ = lat.sign_apply(bt[r:r + 1], KMAX, tol=[TOL], graph=graph)
        ys.append(y)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    y64 = torch.cat(ys).cpu().numpy()
    yb = y32.cpu().numpy()
    diff = max(float(np.linalg.norm(yb[r] - y64[r]) / np.linalg.norm(y64[r])) for r in range(len(ys)))
    lat.close()
    return bt.shape[0] / dt, diff


def plain_fp64_single(ovs, torch, dev, U, bt, k_used, y32, nsrc=NRHS, mu=MU):
    """The plain single-source FP64 form of the same solve: one source at a
    time, each two-sided Lanczos step (Section 4) as separate launches -- the
    library's FP64 stencil for A v and A^dag w (ovs_apply, canonical layout),
    torch dot / norm / axpy kernels, the scalars through the host -- with the
    basis kept, the library's inner sign of G_k and y = |b| V x; no fusion,
    no batching, no graphs.  k = the batched run's k_used for the source, so
    both reach the same accuracy.  Timed on the first nsrc sources; returns
    solves/s and the largest relative difference from the batched result."""
    lat = ovs.Lattice(DIMS, precision="f64")
    lat.set_links(U)
    lat.set_params(MW, mu)

    def solve(b, k):
        nb = torch.linalg.vector_norm(b)
        v = b / nb
        w = v.clone()
        V = torch.empty((k, b.numel()), dtype=torch.complex128, device=dev)
        al, be, ga = [], [], []
        v0 = w0 = None
        for i in range(k):
            V[i] = v
            t = lat.apply("A", v)
            a = torch.vdot(w, t).item()
            al.append(a)
            if i == k - 1:
                break
            sv = lat.apply("A_dag", w)
            vt = t - a * v
            wt = sv - np.conj(a) * w
            if i > 0:
                vt = vt - ga[-1] * v0
                wt = wt - np.conj(be[-1]) * w0
            bn = torch.linalg.vector_norm(vt).item()
            g = torch.vdot(wt, vt).item() / bn
            be.append(bn)
            ga.append(g)
            v0, w0 = v, w
            v = vt / bn
            w = wt / np.conj(g)
        x, _ = lat.inner_sign_tridiag(np.array(al), np.array(be + [0.0]), np.array(ga + [0.0]))
        return nb * (torch.from_numpy(x[0]).to(dev) @ V)

    solve(bt[0], 20)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ys = [solve(bt[r], int(k_used[r])) for r in range(nsrc)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    yb = y32.cpu().numpy()
    diff = max(float(np.linalg.norm(yb[r] - ys[r].cpu().numpy()) / np.linalg.norm(ys[r].cpu().numpy()))
               for r in range(nsrc))
    lat.close()
    return nsrc / dt, diff


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP64 single-source comparison")
    ap.add_argument("--stencil-only", action="store_true",
                    help="time the stencil kernel only (for counter collection)")
    ap.add_argument("--tuning", default=SAVED_TUNING,
                    help="JSON file with a saved kernel configuration: loaded if present, "
                         "written after autotuning otherwise (default: the configuration "
                         "the autotuner chose on an MI355X, the one the committed counter "
                         "profiles were taken with)")
    ap.add_argument("--retune", action="store_true",
                    help="autotune even if the tuning file holds a configuration")
    ap.add_argument("--gradient-only", nargs="+", metavar="ARG", default=None,
                    help="LXxLYxLZxLT K [M]: only time the gradient (ovs_sign_apply_vjp) "
                         "against the forward on that lattice at k iterations, with M computed "
                         "eigentriples if given (for profiling), e.g. 8x8x8x8 400 30")
    ap.add_argument("--eig-only", nargs=4, metavar=("LXxLYxLZxLT", "M", "EPS", "MU"), default=None,
                    help="only time ovs_deflation_compute (m eigentriples, FP64, tol 1e-10) on "
                         "that lattice; prints one JSON line")
    ap.add_argument("--config5-only", action="store_true",
                    help="only run the 16^3 x 32 eps 0.8 mu 0.1 deflated configuration; one JSON line")
    ap.add_argument("--methods-only", action="store_true",
                    help="only run the 2sL-against-Arnoldi comparison at 8^4; prints one JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device to device 5 times: the known-size reference "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; --gpus above 1 is not supported"}))
        sys.exit(2)

    if args.config5_only:
        import torch
        import paper_0810_4228_amd as ovs
        print(json.dumps(config5(ovs, torch, torch.device("cuda:0"))))
        return
    if args.methods_only:
        import torch
        import paper_0810_4228_amd as ovs
        print(json.dumps(compare_methods(ovs, torch, torch.device("cuda:0"))))
        return
    if args.eig_only:
        import torch
        import paper_0810_4228_amd as ovs
        dims = tuple(int(x) for x in args.eig_only[0].split("x"))
        print(json.dumps(eig_timing(ovs, torch, torch.device("cuda:0"), dims=dims,
                                    eps=float(args.eig_only[2]), mu=float(args.eig_only[3]),
                                    m=int(args.eig_only[1]))))
        return
    if args.gradient_only:
        import torch
        import paper_0810_4228_amd as ovs
        dims = tuple(int(x) for x in args.gradient_only[0].split("x"))
        mdef = int(args.gradient_only[2]) if len(args.gradient_only) > 2 else 0
        print(json.dumps(gradient_timing(ovs, torch, torch.device("cuda:0"), dims=dims,
                                         k=int(args.gradient_only[1]), m_defl=mdef)))
        return
    cpu_t = None
    if not args.no_cpu and not args.stencil_only and not args.copy_calibration:
        log(f"bench: cpu baseline ({CPU_PROCS} oracle processes, before GPU use)")
        cpu_t = cpu_oracle_timing()
        log(f"bench: cpu oracle {cpu_t[0]:.3f} s per iteration per process")

    import torch

    if args.copy_calibration:
        n = 256 * 1024 * 1024 // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": 4 * n, "dispatches": 5}))
        return

    import paper_0810_4228_amd as ovs
    import synth

    dev = torch.device("cuda:0")
    V = synth.volume(DIMS)
    log("bench: building inputs", DIMS)
    U = synth.random_links(DIMS, EPS, seed=synth.LINK_SEED)
    b = synth.gaussian_sources(DIMS, NRHS, seed=synth.SOURCE_SEED)
    lat = ovs.Lattice(DIMS, precision="f32")
    Ut = torch.from_numpy(U).to(dev)
    lat.set_links(Ut)
    lat.set_params(MW, MU)
    bt = torch.from_numpy(b).to(dev)
    del U
    key = f"{DIMS}-{NRHS}-f32"
    saved = None
    if args.tuning and os.path.exists(args.tuning) and not args.retune:
        with open(args.tuning) as fh:
            saved = json.load(fh).get(key)
    if saved:
        log("bench: tuning from", args.tuning)
        lat.set_tuning_raw(NRHS, saved)
        tuning_src = "saved: " + os.path.relpath(args.tuning, ROOT)
    else:
        log("bench: autotune")
        lat.autotune(NRHS)
        tuning_src = "autotuned in this run"
        if args.tuning and args.tuning != SAVED_TUNING:
            with open(args.tuning, "w") as fh:
                json.dump({key: lat.get_tuning_raw(NRHS)}, fh)
    rb, wg = lat.get_tuning(NRHS)
    tuning = lat.get_tuning_ex(NRHS)
    log("bench: tuning", tuning)

    # ---- stencil kernel (resident fields, library stream, HIP events) ----
    fi, fo = lat.field_create(NRHS), lat.field_create(NRHS)
    fi.import_(bt)
    fi.apply_timed("A", fo, 20)
    ms_st = fi.apply_timed("A", fo, 200)
    es = 8
    st_bytes = stencil_bytes(V, NRHS, es)
    st_gbs = st_bytes / (ms_st * 1e-3) / 1e9
    log(f"bench: stencil {ms_st * 1e3:.1f} us/apply, {st_gbs:.0f} GB/s (block {rb}, wg {wg})")
    # ---- dual stencil of the Lanczos step: the solve's dominant kernel ----
    fi.dual_timed(20)
    ms_du = fi.dual_timed(200)
    du_bytes = dual_bytes(V, NRHS, es)
    du_gbs = du_bytes / (ms_du * 1e-3) / 1e9
    du_name = dual_kernel_name(tuning["dual"])
    log(f"bench: dual stencil {du_name} {ms_du * 1e3:.1f} us/apply, {du_gbs:.0f} GB/s")
    fi.close()
    fo.close()

    if args.stencil_only:
        print(json.dumps({"stencil_us": ms_st * 1e3, "stencil_gbps": st_gbs,
                          "dual_us": ms_du * 1e3, "dual_gbps": du_gbs, "tuning": tuning}))
        return

    copy_gbs = copy_bandwidth(torch, dev)
    log(f"bench: device copy {copy_gbs:.0f} GB/s")

    # ---- sign solves ----
    tol = [TOL] * NRHS
    for w in range(args.warmup):
        log("bench: warmup step", w)
        y, info, st = lat.sign_apply(bt, KMAX, tol=tol, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for s in range(args.steps):
        y, info, st = lat.sign_apply(bt, KMAX, tol=tol, graph=True)
        infos.append(info)
        log("bench: step", s, "k_used", [i["k_used"] for i in info])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    solves = NRHS * args.steps
    value = solves / dt
    last = infos[-1]
    k_used = [i["k_used"] for i in last]
    k_avg = float(np.mean(k_used))
    est = max(i["est_rel_err"] for i in last)
    phase = {k: last[0][k] for k in ("t_defl_ms", "t_krylov_ms", "t_inner_ms", "t_combine_ms")}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "sgn(gamma5 Dw(mu)) b by two-sided Lanczos, 16^3x32, 12 Gaussian sources",
            "lattice": "16x16x16x32",
            "links": "P_SU3(1+0.6G) seed 0",
            "m_w": MW, "mu": MU, "nrhs": NRHS, "tol": TOL, "k_max": KMAX, "n_defl": 0,
            "storage": "f32 vectors and links, f64 coefficients/dots",
            "graph": True,
        },
        "tuning": tuning,
        "tuning_source": tuning_src,
        # caller-workspace requirement (the k_max layout) and what the handle
        # actually holds after the timed solves (basis grown as needed)
        "workspace_bytes": lat.workspace_size(NRHS, KMAX),
        "workspace_held_bytes": lat.workspace_held(),
        "k_used": k_used,
        "est_rel_err_max": est,
        "phase_ms": phase,
        "stencil": {"kernel": "k_wilson<float>", "us_per_apply": ms_st * 1e3, "gbps": st_gbs,
                    "frac_peak": st_gbs / HBM_PEAK_GBS, "rhs_block": rb, "wg": wg,
                    "staged_tile": tuning["stencil"]["staged_tile"],
                    "bytes_per_apply": st_bytes, "traffic": measured_traffic("stencil", tuning)},
        "dual_stencil": {"kernel": du_name, "us_per_apply": ms_du * 1e3, "gbps": du_gbs,
                         "frac_peak": du_gbs / HBM_PEAK_GBS, "bytes_per_apply": du_bytes},
        "roofline": {"bound": "hbm", "kernel": du_name, "achieved": du_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": du_gbs / HBM_PEAK_GBS,
                     "traffic": measured_traffic("dual", tuning),
                     "copy_gbps": copy_gbs, "frac_of_copy": du_gbs / copy_gbs},
    }
    if not args.no_compare:
        log("bench: FP64 single-source comparison")
        cmp = {}
        for graph in (False, True):
            rate, diff = fp64_single_source(ovs, torch, dev, Ut, bt, y, graph)
            key = "fp64_single_graph" if graph else "fp64_single"
            cmp[key] = {"solves_per_s": rate, "ratio": value / rate, "max_rel_diff_vs_batched": diff}
            log(f"bench: {key}: {rate:.2f} solves/s, batched/this = {value / rate:.2f}")
        rate, diff = plain_fp64_single(ovs, torch, dev, Ut, bt, k_used, y)
        cmp["plain_fp64_single"] = {"solves_per_s": rate, "ratio": value / rate,
                                    "max_rel_diff_vs_batched": diff, "sources_timed": NRHS,
                                    "form": "one source, FP64, unfused launches, host scalars, no graph, k = k_used"}
        log(f"bench: plain_fp64_single: {rate:.2f} solves/s, batched/this = {value / rate:.2f}")
        # the same three forms at the other chemical potential of the comparison
        lat01 = ovs.Lattice(DIMS, precision="f32")
        lat01.set_links(Ut)
        lat01.set_params(MW, 0.1)
        lat01.set_tuning_raw(NRHS, lat.get_tuning_raw(NRHS))
        lat01.sign_apply(bt, KMAX, tol=[TOL] * NRHS, graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            y01, info01, _ = lat01.sign_apply(bt, KMAX, tol=[TOL] * NRHS, graph=True)
        torch.cuda.synchronize()
        v01 = 3 * NRHS / (time.perf_counter() - t0)
        k01 = [i["k_used"] for i in info01]
        lat01.close()
        r64, d64 = fp64_single_source(ovs, torch, dev, Ut, bt, y01, True, mu=0.1)
        rpl, dpl = plain_fp64_single(ovs, torch, dev, Ut, bt, k01, y01, mu=0.1)
        cmp["mu_0.1"] = {"batched_solves_per_s": v01, "k_used": k01,
                         "fp64_single_graph": {"solves_per_s": r64, "ratio": v01 / r64,
                                               "max_rel_diff_vs_batched": d64},
                         "plain_fp64_single": {"solves_per_s": rpl, "ratio": v01 / rpl,
                                               "max_rel_diff_vs_batched": dpl}}
        log(f"bench: mu 0.1: batched {v01:.2f} solves/s, x{v01 / r64:.2f} fused FP64, "
            f"x{v01 / rpl:.2f} plain FP64")
        out["vs_fp64_single_source"] = cmp
    if not args.no_compare:
        log("bench: launch modes")
        out["launch_modes"] = launch_modes(ovs, torch, dev, lat, bt)
        log("bench: launch modes", out["launch_modes"])
    if not args.no_compare:
        log("bench: gradient timing")
        out["gradient"] = [gradient_timing(ovs, torch, dev),
                           gradient_timing(ovs, torch, dev, dims=(16, 16, 16, 16), k=200),
                           gradient_timing(ovs, torch, dev, m_defl=30)]
        log("bench: config 5 (eps 0.8, mu 0.1, mixed tolerances, 40 eigentriples)")
        out["config5"] = config5(ovs, torch, dev)
        log("bench: config5", out["config5"])
        log("bench: 2sL against Arnoldi")
        out["methods"] = compare_methods(ovs, torch, dev)
        log("bench: methods", out["methods"])
        log("bench: overlap eigenvalues")
        out["overlap_eigs"] = overlap_eigs_timing(ovs, torch, dev)
        log("bench: gradient", out["gradient"])
    if not args.no_check:
        log("bench: free-field accuracy check")
        err, kf = free_field_check(ovs, torch, dev)
        out["rel_err_free_field"] = err
        out["free_field_k_used"] = kf
    if cpu_t is not None:
        out["cpu_baseline"] = cpu_baseline(cpu_t[0], cpu_t[1], k_avg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
