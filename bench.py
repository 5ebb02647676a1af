"""Time-to-solution and preconditioner throughput of the FlashMP hot path on one GPU.

Workload: 256^3 Yee grid with PEC walls, 8 x 8 x 8 subdomains of 32^3 cells
(overlap 1), eps_r ~ U[1,10] on 8^3-cell cubes, c = 2, right-hand side N(0,1)
(seed 3).  One step = one full FGMRES(30) solve in FP64 to a relative residual
of 1e-8 from x0 = 0, with the FlashMP RAS preconditioner (FP64 transforms).
Variants (FP32 transforms) are timed the same way and reported beside it.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("time-to-solution at rel. residual 1e-8 (256³) + precond applies/s; "
          "plain vs mixed/learned")
HBM_PEAK_GBS = 8000.0

# HBM traffic of each roofline kernel as a multiple of its algorithmic bytes,
# from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this bench on the 256^3
# workload (KiB per dispatch, scaled by what the counters read for a plain
# device copy of one vector: FETCH x2.000, WRITE x1.000).  A ratio holds only
# for the kernel sources it was measured on: if any listed source changed
# since, traffic is null.
TRAFFIC = {
    "k_mupdate": (1.0000, {"fmp_krylov.hip": "2d8ce5abd17a3d4d663922d953a4ffdb81ffb46d83ff33b0d1ea22998bc560f2",
                          "fmp_common.h": "29e6d322f7b76d24dd01922e0bcf5b2fd956d45b445f79172e6746defd9f6869"}),
    "k_mdot": (1.0001, {"fmp_krylov.hip": "2d8ce5abd17a3d4d663922d953a4ffdb81ffb46d83ff33b0d1ea22998bc560f2",
                        "fmp_common.h": "29e6d322f7b76d24dd01922e0bcf5b2fd956d45b445f79172e6746defd9f6869"}),
    # per stencil tile height (halo rows re-read through L2 differ by tile)
    "k_curlcurl": ({4: 1.0413, 8: 1.0322, 16: 1.0328}, {"fmp_stencil.hip": "696e04ec48a51593d192077df34e99a631009e7660df29edde94fb7fbba8ea32",
                            "fmp_common.h": "29e6d322f7b76d24dd01922e0bcf5b2fd956d45b445f79172e6746defd9f6869"}),
    # the three passes of one apply over the algorithmic 16 B per unknown
    "precond_apply": (3.5960, {"fmp_transform.hip": "451b2ffc4bca4d36a132b61d611652d0d7c2de1e1144a15cd2ff955cf703e5ac",
                               "fmp_api.hip": "7115c5d95370c97565f6ce717e935680f02323ad55970b187b67041eca2ca2a6",
                               "fmp_common.h": "29e6d322f7b76d24dd01922e0bcf5b2fd956d45b445f79172e6746defd9f6869"}),
}


FP64_VECTOR_PEAK_TFLOPS = 78.6


def transform_flops_per_apply(n, sub, overlap=1):
    """FP64 flops of one preconditioner apply's transforms on an n^3 grid cut
    into sub^3 subdomains (boxes = owned block + overlap, clipped at walls):
    per box, component and axis, every pencil along that axis is contracted
    forward and back with the even/odd butterfly, n_axis^2 / 2 FMAs each way."""
    def sides(nn, s):
        out = []
        for a in range(0, nn, s):
            out.append(min(nn, a + s + overlap) - max(0, a - overlap))
        return out
    sx = sides(n, sub[0]); sy = sides(n, sub[1]); sz = sides(n, sub[2])
    fma = 0
    for bz in sz:
        for by in sy:
            for bx in sx:
                for (na, other) in ((bx, by * bz), (by, bx * bz), (bz, bx * by)):
                    fma += 3 * other * (na * na / 2.0) * 2      # 3 components, forward + inverse
    return 2.0 * fma


def traffic_ratio(name, variant=None):
    import hashlib
    if name not in TRAFFIC:
        return None
    ratio, srcs = TRAFFIC[name]
    if isinstance(ratio, dict):
        ratio = ratio.get(variant)
        if ratio is None:
            return None
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2508_07193_amd", "csrc")
    for f, h in srcs.items():
        try:
            with open(os.path.join(d, f), "rb") as fh:
                if hashlib.sha256(fh.read()).hexdigest() != h:
                    return None
        except OSError:
            return None
    return ratio


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(P, iters, sample_boxes=512, reps=4):
    """Time the CPU oracle on a bounded sample of one FGMRES iteration's work and scale it.

    Sample: `reps` passes over `sample_boxes` of the 512 subdomain solves
    (all of them by default: one whole preconditioner apply per pass), ten
    sparse A x on a 64^3 sub-grid (scaled by unknown count), and twenty dots
    and axpys on full 256^3 vectors (scaled to the CGS work of an average
    Arnoldi step, j = 15: 2j + 5 vector passes); about 10-20 s of CPU work.
    Reported as the estimated time-to-solution for the same iteration count
    as the GPU run; `cores` is the BLAS thread count the oracle's numpy calls
    use.
    """
    from oracle import ras, yee
    cores = blas_threads()
    n = P["nx"]
    eps_cell = yee.expand_eps(P["eps"], P["eps_block"], n, n, n)
    nsub = (n // P["sub"][0]) ** 3
    which = list(np.linspace(0, nsub - 1, sample_boxes).astype(int))
    t0 = time.perf_counter()
    for _ in range(reps):
        ras.ras_apply_subset(P["rhs"], P["c"], P["sub"], 1, eps_cell, which)
    m_pre = time.perf_counter() - t0
    t_pre = m_pre / reps * nsub / sample_boxes
    m = 64
    A = yee.assemble_A(m, m, m, P["c"], eps_cell[:m, :m, :m])
    xs = yee.from_padded(P["rhs"][:, :m, :m, :m])
    t0 = time.perf_counter()
    for _ in range(10):
        A @ xs
    m_spmv = time.perf_counter() - t0
    t_spmv = m_spmv / 10 * (yee.n_unknowns(n, n, n) / xs.size)
    a = P["rhs"].ravel()
    b = np.roll(a, 1)
    t0 = time.perf_counter()
    for _ in range(20):
        float(np.dot(a, b))
        c = a + 0.5 * b
    m_vec = time.perf_counter() - t0
    t_vec = m_vec / 40
    del c
    per_it = t_pre + t_spmv + (2 * 15 + 5) * t_vec
    total = per_it * iters
    out = dict(value=round(total * 1e3, 1), unit="ms", cores=cores, kind="oracle",
               sample=(f"{reps} x {sample_boxes}/{nsub} subdomain solves (a whole preconditioner "
                       f"apply each), ten 64^3 sparse A x, twenty dots and axpys on 256^3 vectors, "
                       f"scaled to {iters} FGMRES iterations ({per_it * 1e3:.0f} ms per iteration); "
                       f"the whole 128^3 solve is measured end to end in cpu_oracle_c2"),
               seconds_measured=round(m_pre + m_spmv + m_vec, 2))
    out.update(cpu_info())
    return out


def cpu_info():
    """Host CPU model (from /proc/cpuinfo) and the logical CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count()
    return dict(cpu_model=model, nproc=ncpu)


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count()


def cpu_oracle_c2():
    """The CPU oracle's full solve of the 128^3 workload, measured end to end:
    sparse assembly of A, then right-preconditioned BiCGSTAB in FP64 to 1e-8
    with the oracle's RAS (every subdomain solved by the transform route of
    oracle.transforms).  Returns the timings and the solution (padded)."""
    from oracle import krylov, ras, yee
    from paper_2508_07193_amd import inputs
    P = inputs.make_problem("c2")
    n = P["nx"]
    eps_cell = yee.expand_eps(P["eps"], P["eps_block"], n, n, n)
    t0 = time.perf_counter()
    A = yee.assemble_A(n, n, n, P["c"], eps_cell)
    t_asm = time.perf_counter() - t0

    def Aop(v):
        return yee.to_padded(A @ yee.from_padded(v), n, n, n)

    def Mop(v):
        return ras.ras_apply(v, P["c"], P["sub"], 1, eps_cell)
    t0 = time.perf_counter()
    x, info = krylov.bicgstab(Aop, P["rhs"], M=Mop, tol=P["tol"], maxiter=500)
    t_solve = time.perf_counter() - t0
    t0 = time.perf_counter()
    Mop(P["rhs"])
    t_pre = time.perf_counter() - t0
    out = dict(kind="oracle", measured="whole solve", time_to_solution_s=round(t_solve, 2),
               assembly_s=round(t_asm, 2), iterations=int(info["iterations"]),
               rel_residual_true=float(info["rel_true"]),
               precond_applies_per_s=round(1.0 / t_pre, 3), threads=blas_threads(),
               workload="128^3, 4^3 subdomains of 32^3 (overlap 1), eps_r U[1,10] on 8^3 cubes, "
                        "c=2, RHS N(0,1) seed 2; BiCGSTAB FP64 to 1e-8 (CPU oracle, NumPy/SciPy)")
    out.update(cpu_info())
    return out, x


def c2_leg(args, dev, log):
    """128^3 workload (4^3 subdomains of 32^3, eps_r U[1,10] on 8^3 cubes, c = 2,
    seed 2): BiCGSTAB in FP64 to 1e-8 with the FP64 FlashMP RAS (the configured
    solver), and FGMRES(30) in FP64 with FP32 and BF16 transforms on the same
    grid.  Solutions are written to args.c2_dir for the comparison with the CPU
    oracle's solution in the parent process."""
    import torch
    from paper_2508_07193_amd import api, inputs
    P = inputs.make_problem("c2")
    n = P["nx"]
    dom = dict(nx=n, ny=n, nz=n, c=P["c"], eps=P["eps"], eps_block=P["eps_block"], sub=P["sub"])
    b = torch.from_numpy(P["rhs"].ravel()).to(dev)
    res = {}
    for prec, solver in (("fp64", "bicgstab"), ("fp32", "fgmres"), ("bf16", "fgmres")):
        h = api.Handle([dom], overlap=1, precision=prec, device=dev, use_graph=args.graphs,
                       batch_boxes=-1)
        h.autotune(b)
        x = h.new_vector()
        kw = dict(solver=solver, rtol=P["tol"], max_iter=500)
        for _ in range(max(1, args.warmup)):
            x.zero_()
            h.solve(b, x, **kw)
        times = []
        for _ in range(max(1, args.steps)):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = h.solve(b, x, **kw)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        z = h.new_vector()
        h.apply_precond(b, z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            h.apply_precond(b, z)
        torch.cuda.synchronize()
        t_pre = (time.perf_counter() - t0) / 20 * 1e3
        if args.c2_dir:
            np.save(os.path.join(args.c2_dir, f"x_{prec}.npy"), x.cpu().numpy())
        res[prec] = dict(solver=solver, transforms=prec, time_to_solution_ms=round(float(np.mean(times)), 2),
                         iterations=info["iterations"], rel_residual_true=info["rel_residual_true"],
                         n_precond=info["n_precond"], n_spmv=info["n_spmv"],
                         precond_ms=round(t_pre, 4), precond_applies_per_s=round(1e3 / t_pre, 1))
        log(f"[c2] {prec} {solver}: {res[prec]}")
        h.close()
    return dict(workload="128^3 Yee grid, PEC walls, 4^3 subdomains of 32^3 (overlap 1), eps_r "
                         "U[1,10] on 8^3 cubes, c=2, RHS N(0,1) seed 2; FP64 Krylov to 1e-8",
                runs=res)


def learned_leg(args, dev, log):
    """256^3, c = 8: FGMRES with and without the trained coarse correction.

    Pairs: args.pairs_rhs right-hand sides (seeds 1005+) x args.pairs_per_rhs
    FGMRES iterates; held-out right-hand sides: seeds 2005..2009.
    """
    import torch
    from paper_2508_07193_amd import api, inputs, learned
    P = inputs.make_problem("c5")
    n = P["nx"]
    dom = dict(nx=n, ny=n, nz=n, c=P["c"], eps=P["eps"], eps_block=P["eps_block"], sub=P["sub"])
    h = api.Handle([dom], overlap=1, precision="fp64", use_learned=True, device=dev,
                   batch_boxes=-1, use_graph=args.graphs)
    h.autotune()
    t0 = time.perf_counter()
    X, Y = learned.generate_pairs(h, (n, n, n), args.pairs_rhs, args.pairs_per_rhs, 1005, log=log)
    t_pairs = time.perf_counter() - t0
    t0 = time.perf_counter()
    params, hist = learned.train(X, Y, hidden=256, epochs=args.epochs, batch=100, lr=1e-3,
                                 device=dev, log=log)
    t_train = time.perf_counter() - t0
    res = {"plain": [], "learned": []}
    x = h.new_vector()
    for mode in ("plain", "learned"):
        api.fmp_set_coarse_model(h, 256, params if mode == "learned" else None)
        for sd in range(2005, 2010):
            b = torch.from_numpy(inputs.extra_rhs(n, n, n, sd).ravel()).to(dev)
            x.zero_()
            h.solve(b, x, solver="fgmres", rtol=1e-8, max_iter=500)      # warm
            x.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            info = h.solve(b, x, solver="fgmres", rtol=1e-8, max_iter=500)
            torch.cuda.synchronize()
            info["wall_ms"] = (time.perf_counter() - t1) * 1e3
            res[mode].append(info)
    it_p = float(np.mean([r["iterations"] for r in res["plain"]]))
    it_l = float(np.mean([r["iterations"] for r in res["learned"]]))
    ms_p = float(np.mean([r["wall_ms"] for r in res["plain"]]))
    ms_l = float(np.mean([r["wall_ms"] for r in res["learned"]]))
    log(f"[learned] plain {it_p} it {ms_p:.1f} ms, learned {it_l} it {ms_l:.1f} ms")
    return dict(workload="256^3, c=8, eps_r U[1,10] 8^3 cubes, FGMRES(30) FP64 to 1e-8; "
                         "held-out RHS seeds 2005-2009",
                pairs=int(X.shape[0]), pair_generation_s=round(t_pairs, 1),
                train_s=round(t_train, 1), final_train_mse=hist[-1], first_epoch_mse=hist[0],
                plain_iterations=it_p, learned_iterations=it_l,
                plain_time_to_solution_ms=round(ms_p, 2), learned_time_to_solution_ms=round(ms_l, 2),
                learned_fallbacks=[r["used_fallback"] for r in res["learned"]],
                learned_rel_residual_true=max(r["rel_residual_true"] for r in res["learned"]),
                speedup_vs_plain=round(ms_p / ms_l, 3))


def batch_leg(args, dev, log):
    """64 independent cubic domains, sides from {24,32,48,64,96}, c ~ U[0.5,8] (seed 4).

    One handle holds all domains; a preconditioner apply covers every box of
    every domain (FP32 transforms) as one hipGraph replay.  The timed solve is
    an independent FGMRES(30) per domain in FP64 to 1e-8, all domains advanced
    in lockstep through shared launches; each domain's residual is recomputed
    here as well.  One FGMRES on the concatenated system is reported beside it.
    """
    import torch
    from paper_2508_07193_amd import api, inputs
    doms_in = inputs.make_batch_c4()
    doms = [dict(nx=d["nx"], ny=d["ny"], nz=d["nz"], c=d["c"], sub=d["sub"]) for d in doms_in]
    h = api.Handle(doms, overlap=1, precision="fp32", device=dev, use_graph=True, batch_boxes=-1)
    b = torch.cat([torch.from_numpy(d["rhs"].ravel()) for d in doms_in]).to(dev)
    n_unk = sum(inputs.n_unknowns(d["nx"], d["ny"], d["nz"]) for d in doms_in)
    z = h.new_vector()
    tune = h.autotune(b, z)
    chosen = [t for t in tune if t["chosen"]][0]
    log(f"[batch] autotune: {[(t['batch_boxes'], t['streams'], t['slab_order'], round(t['apply_ms'], 3)) for t in tune]}")
    h.apply_precond(b, z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        h.apply_precond(b, z)
    torch.cuda.synchronize()
    t_pre = (time.perf_counter() - t0) / 10 * 1e3
    x = h.new_vector()
    y = h.new_vector()

    def timed(per_domain):
        x.zero_()
        h.solve(b, x, solver="fgmres", rtol=1e-8, max_iter=500, per_domain=per_domain)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = h.solve(b, x, solver="fgmres", rtol=1e-8, max_iter=500, per_domain=per_domain)
        torch.cuda.synchronize()
        tts = (time.perf_counter() - t0) * 1e3
        h.curlcurl_apply(x, y)
        rel = []
        for d in range(len(doms)):
            a, e = h.offsets[d], h.offsets[d + 1]
            rel.append(float(torch.linalg.vector_norm(b[a:e] - y[a:e]) / torch.linalg.vector_norm(b[a:e])))
        return info, tts, rel

    info_c, tts_c, rel_c = timed(False)
    info, tts, rel = timed(True)
    its = sorted(info["domain_iterations"])
    sides = [d["nx"] for d in doms_in]
    log(f"[batch] independent: status {info['status']} lockstep steps {info['iterations']}, "
        f"per-domain steps {its}, tts {tts:.1f} ms, max domain rel res {max(rel):.2e}; "
        f"concatenated: {info_c['iterations']} steps, tts {tts_c:.1f} ms, max domain rel res "
        f"{max(rel_c):.2e}; precond {t_pre:.3f} ms")
    return dict(workload="64 cubic domains, sides U{24,32,48,64,96} (seed 4), c ~ U[0.5,8], eps 1; "
                         "FP32 transforms; independent FGMRES(30) per domain, FP64, to 1e-8 each",
                unknowns=n_unk, side_counts={str(k): sides.count(k) for k in sorted(set(sides))},
                time_to_solution_ms=round(tts, 2), lockstep_steps=info["iterations"],
                domain_steps_min_median_max=[its[0], its[len(its) // 2], its[-1]],
                max_domain_rel_residual=max(rel),
                max_domain_rel_residual_solver=max(info["domain_rel_residual"]),
                concatenated_system=dict(time_to_solution_ms=round(tts_c, 2),
                                         iterations=info_c["iterations"],
                                         max_domain_rel_residual=max(rel_c)),
                precond_applies_per_s=round(1e3 / t_pre, 1), precond_ms=round(t_pre, 4),
                autotune=dict(chosen=dict(batch_boxes=chosen["batch_boxes"], streams=chosen["streams"],
                                          slab_order=chosen["slab_order"]),
                              candidates=[[t["batch_boxes"], t["streams"], t["slab_order"],
                                           round(t["apply_ms"], 4)] for t in tune]),
                launch="hipGraph replay of the per-class, per-batch pass sequence")


def convergence_leg(args, dev, log):
    """Shape of the overlap study of Sec. IV (convergence experiments): uniform
    medium, b = A x_rand, stopping at relative residual 1e-12; no
    preconditioner versus RAS with overlap 1, 2, 3 (PEC boxes), and RAS over
    the paper's index blocks with the low-rank boundary correction at overlap
    0 and 1, each under BiCGSTAB and FGMRES(30).  128^3 grid, 4^3 subdomains
    of 32^3, c = 2, FP64 transforms.  (Overlap 0 exists for index blocks
    only: with PEC boxes the interface unknowns would sit on box walls.)"""
    import torch
    from paper_2508_07193_amd import api, inputs
    n, sub, c = 128, 32, 2.0
    xr = torch.from_numpy(inputs.normal_rhs(np.random.default_rng(11), n, n, n).ravel()).to(dev)
    dom = [dict(nx=n, ny=n, nz=n, c=c, sub=(sub, sub, sub))]
    rows = []
    index_setup = {}
    cases = [("pec", g) for g in (0, 1, 2, 3)] + [("index", 0), ("index", 1)]
    for kind, g in cases:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = api.Handle(dom, overlap=g if kind == "index" else max(g, 1), precision="fp64",
                       device=dev, subdomain=kind)
        torch.cuda.synchronize()
        if kind == "index":
            r = xr.clone()
            z = h.new_vector()
            h.apply_precond(r, z)
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            for _ in range(5):
                h.apply_precond(r, z)
            ev1.record()
            torch.cuda.synchronize()
            index_setup[f"overlap{g}"] = dict(
                setup_ms=round((time.perf_counter() - t0) * 1e3, 1),
                apply_ms=round(ev0.elapsed_time(ev1) / 5, 3),
                workspace_gb=round(h.ws.numel() / 1e9, 2))
            log(f"[convergence] index blocks overlap {g}: {index_setup[f'overlap{g}']}")
            del r, z
        b = h.new_vector()
        h.curlcurl_apply(xr, b)
        x = h.new_vector()
        for solver in ("bicgstab", "fgmres"):
            precond = kind == "index" or g > 0
            kw = dict(solver=solver, rtol=1e-12, max_iter=3000, precond=precond)
            x.zero_()
            h.solve(b, x, **kw)
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = h.solve(b, x, **kw)
            torch.cuda.synchronize()
            tts = (time.perf_counter() - t0) * 1e3
            err = float(torch.linalg.vector_norm(x - xr) / torch.linalg.vector_norm(xr))
            name = (f"ras_index_overlap{g}" if kind == "index" else
                    (f"ras_overlap{g}" if g else "none"))
            rows.append(dict(precond=name, solver=solver,
                             iterations=info["iterations"], time_to_solution_ms=round(tts, 2),
                             rel_residual_true=info["rel_residual_true"], rel_err_vs_x_rand=err,
                             status=info["status"]))
            log(f"[convergence] {rows[-1]}")
        h.close()
        del h, b, x
        torch.cuda.empty_cache()
    return dict(workload="128^3 Yee grid, PEC walls, eps 1, c=2, 4^3 subdomains of 32^3, "
                         "b = A x_rand (x_rand N(0,1) seed 11), rel. residual 1e-12",
                rows=rows, index_blocks=index_setup)


def cn_leg(args, dev, log):
    """Crank-Nicolson time stepping around the solve (Sec. II-A, eqs. (2)-(5))
    on the 256^3 medium of the main workload: E^0 = N(0,1) (seed 21), H^0 = 0,
    dt = 2 sqrt(c) = 2 sqrt(2); each step builds R, solves A E+ = R by FP64
    FGMRES(30) with the FP64 RAS to 1e-8 of the warm-start residual, and
    updates H.  Reports time per step, iterations and the drift of the
    discrete energy (1/2)(E^T eps E + H^T H), which Crank-Nicolson conserves
    up to the solve tolerance."""
    import torch
    from paper_2508_07193_amd import api, inputs
    P = inputs.make_problem(args.config)
    n, blk = P["nx"], P["eps_block"]
    h = api.Handle([dict(nx=n, ny=n, nz=n, c=P["c"], eps=P["eps"], eps_block=blk, sub=P["sub"])],
                   precision="fp64", device=dev)
    cell = torch.from_numpy(P["eps"]).to(dev)
    for ax in range(3):
        cell = cell.repeat_interleave(blk, dim=ax)
    ee = torch.zeros(3, n, n, n, dtype=torch.float64, device=dev)      # edge eps, padded
    ee[0, 1:, 1:, :] = 0.25 * (((cell[:-1, :-1, :] + cell[1:, :-1, :]) + cell[:-1, 1:, :]) + cell[1:, 1:, :])
    ee[1, 1:, :, 1:] = 0.25 * (((cell[:-1, :, :-1] + cell[1:, :, :-1]) + cell[:-1, :, 1:]) + cell[1:, :, 1:])
    ee[2, :, 1:, 1:] = 0.25 * (((cell[:, :-1, :-1] + cell[:, 1:, :-1]) + cell[:, :-1, 1:]) + cell[:, 1:, 1:])
    ee = ee.reshape(-1)
    del cell
    E = torch.from_numpy(inputs.normal_rhs(np.random.default_rng(21), n, n, n).ravel()).to(dev)
    H = h.new_vector()

    def energy():
        return 0.5 * float(torch.dot(ee * E, E) + torch.dot(H, H))

    W0 = energy()
    kw = dict(solver="fgmres", rtol=1e-8, max_iter=300)
    h.cn_step(E, H, **kw)                                # warm-up step (not timed)
    steps, its, drift = max(3, args.steps), [], []
    W = energy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = h.cn_step(E, H, **kw)
        its.append(info["iterations"])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    W1 = energy()
    log(f"[cn] {steps} steps, {ms:.2f} ms/step, iterations {its}, energy {W0:.6e} -> {W:.6e} -> {W1:.6e}")
    return dict(workload="256^3 Yee grid, PEC walls, eps_r U[1,10] on 8^3 cubes, c=2 (dt = 2 sqrt(2)), "
                         "E0 N(0,1) seed 21, H0 = 0; FP64 FGMRES(30) + FP64 RAS to 1e-8 of the "
                         "warm-start residual per step",
                steps_timed=steps, ms_per_step=round(ms, 2), iterations_per_step=its,
                energy_rel_drift_per_step=abs(W1 - W) / W / steps,
                energy_rel_drift_total=abs(W1 - W0) / W0)


def whole_leg(args, dev, log):
    """The 64 uneven domains of the batch leg solved with one box per domain
    (sides up to 96: the size classes 64 and 96, as matrix-core GEMMs in BF16
    or tiled vector-ALU GEMMs in FP32): the preconditioner is each domain's
    exact inverse up to the transform rounding.  Independent FGMRES(30) per
    domain in FP64 to 1e-8, lockstep, hipGraph replay of the applies."""
    import torch
    from paper_2508_07193_amd import api, inputs
    prec = args.prec or "bf16"
    doms_in = inputs.make_batch_c4()
    doms = [dict(nx=d["nx"], ny=d["ny"], nz=d["nz"], c=d["c"], sub=(0, 0, 0)) for d in doms_in]
    h = api.Handle(doms, overlap=1, precision=prec, device=dev, use_graph=True, batch_boxes=-1)
    b = torch.cat([torch.from_numpy(d["rhs"].ravel()) for d in doms_in]).to(dev)
    z = h.new_vector()
    tune = h.autotune(b, z)
    h.apply_precond(b, z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        h.apply_precond(b, z)
    torch.cuda.synchronize()
    t_pre = (time.perf_counter() - t0) / 10 * 1e3
    x, y = h.new_vector(), h.new_vector()
    h.solve(b, x, solver="fgmres", rtol=1e-8, max_iter=100, per_domain=True)
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = h.solve(b, x, solver="fgmres", rtol=1e-8, max_iter=100, per_domain=True)
    torch.cuda.synchronize()
    tts = (time.perf_counter() - t0) * 1e3
    h.curlcurl_apply(x, y)
    rel = []
    for d in range(len(doms)):
        a, e = h.offsets[d], h.offsets[d + 1]
        rel.append(float(torch.linalg.vector_norm(b[a:e] - y[a:e]) / torch.linalg.vector_norm(b[a:e])))
    its = sorted(info["domain_iterations"])
    log(f"[whole {prec}] lockstep {info['iterations']}, per-domain {its}, tts {tts:.1f} ms, "
        f"max domain rel res {max(rel):.2e}, precond {t_pre:.3f} ms")
    chosen = [t for t in tune if t["chosen"]][0]
    kind = ("BF16 transforms on the matrix cores" if prec == "bf16" else
            f"{prec.upper()} transforms (tiled GEMMs for sides above 48)")
    return dict(workload=f"the 64 domains of batch_c4, one box per domain (sides 24..96), {kind}; "
                         "independent FGMRES(30) per domain, FP64, to 1e-8 each",
                time_to_solution_ms=round(tts, 2), lockstep_steps=info["iterations"],
                domain_steps_min_median_max=[its[0], its[len(its) // 2], its[-1]],
                max_domain_rel_residual=max(rel), precond_ms=round(t_pre, 4),
                precond_applies_per_s=round(1e3 / t_pre, 1),
                autotune_chosen=dict(batch_boxes=chosen["batch_boxes"], streams=chosen["streams"],
                                     slab_order=chosen["slab_order"]))


def c3_context(args):
    """Problem, device vectors and timing helpers of the 256^3 legs (child process)."""
    import torch
    from paper_2508_07193_amd import api, inputs

    dev = "cuda:0"
    torch.cuda.set_device(0)
    P = inputs.make_problem(args.config)
    n = P["nx"]
    dom = dict(nx=n, ny=n, nz=n, c=P["c"], eps=P["eps"], eps_block=P["eps_block"], sub=P["sub"])
    b = torch.from_numpy(P["rhs"].ravel()).to(dev)
    n_unk = inputs.n_unknowns(n, n, n)
    stream = torch.cuda.current_stream()

    def run_solves(h, steps, warmup, tag):
        x = h.new_vector()
        info = None
        for _ in range(warmup):
            x.zero_()
            info = h.solve(b, x, solver="fgmres", restart=30, rtol=1e-8, max_iter=500)
        torch.cuda.synchronize()
        times = []
        for _ in range(steps):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = h.solve(b, x, solver="fgmres", restart=30, rtol=1e-8, max_iter=500)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        log(f"[{tag}] solve: {info}  ms={times}")
        return x, info, float(np.mean(times))

    def time_events(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    def tuned_handle(prec):
        hh = api.Handle([dom], overlap=1, precision=prec, device=dev, batch_boxes=-1,
                        use_graph=args.graphs)
        t = hh.autotune(b)
        c = [e for e in t if e["chosen"] and not e["stencil_ty"]][0]
        ty = [e["stencil_ty"] for e in t if e["chosen"] and e["stencil_ty"]]
        log(f"[{prec}] autotune: {[(e['batch_boxes'], e['streams'], e['slab_order'], e['stencil_ty'], round(e['apply_ms'], 4)) for e in t]}")
        return hh, dict(batch_boxes=c["batch_boxes"], streams=c["streams"], slab_order=c["slab_order"],
                        graph=bool(args.graphs), stencil_ty=ty[0] if ty else None)

    return dict(torch=torch, P=P, b=b, n_unk=n_unk, run_solves=run_solves,
                time_events=time_events, tuned_handle=tuned_handle)


def main_leg(args):
    """Plain FP64 FlashMP on the 256^3 workload: the bench value, rooflines, calibration."""
    C = c3_context(args)
    torch, b, n_unk = C["torch"], C["b"], C["n_unk"]
    time_events = C["time_events"]
    h, plan64 = C["tuned_handle"]("fp64")
    log(f"handle ready: workspace {h.ws.numel() / 2**20:.0f} MiB, vector {h.length} doubles")
    x64, info64, tts64 = C["run_solves"](h, args.steps, args.warmup, "fp64")
    z = h.new_vector()
    y = h.new_vector()
    t_pre = time_events(lambda: h.apply_precond(b, z), 10)
    t_spmv = time_events(lambda: h.curlcurl_apply(b, y), 20)

    def roof(name, kernel, bytes_per_launch, avg_ms, per, variant=None):
        ach = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        ratio = traffic_ratio(name, variant)
        return dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 3),
                    traffic=None if ratio is None else round(ratio * bytes_per_launch),
                    kernel=kernel,
                    bytes_per_launch=round(bytes_per_launch), avg_ms=round(avg_ms, 4),
                    algorithmic_bytes=per)

    # one more solve with the library's event timing of each kernel class
    x = h.new_vector()
    pinfo = h.solve(b, x, solver="fgmres", restart=30, rtol=1e-8, max_iter=500, profile=True)
    log(f"[fp64 profiled] {pinfo}")
    spmv_bytes = 16.0 * n_unk
    roofs = {
        "k_mupdate": roof("k_mupdate", "k_mupdate (CGS: w -= V h, ||w||^2)",
                          pinfo["bytes_orth_update"] / pinfo["n_orth_update"],
                          pinfo["t_orth_update_ms"] / pinfo["n_orth_update"],
                          "8 B x len x (j+2) per launch (reads V_0..V_j and w, writes w)"),
        "k_mdot": roof("k_mdot", "k_mdot (CGS: h = V^T w, ||w||^2)",
                       pinfo["bytes_orth_dot"] / pinfo["n_orth_dot"],
                       pinfo["t_orth_dot_ms"] / pinfo["n_orth_dot"],
                       "8 B x len x (j+2) per launch (reads V_0..V_j and w)"),
        "k_curlcurl": roof("k_curlcurl", f"k_curlcurl (stencil y = A x, 64 x {plan64['stencil_ty']} tiles)",
                           spmv_bytes, t_spmv, "16 B per unknown (x in, y out)",
                           variant=plan64["stencil_ty"]),
        "precond_apply": roof("precond_apply", "precond apply (passes A, B, C)", 16.0 * n_unk, t_pre,
                              "16 B per unknown (r in, z out); staging traffic excluded"),
    }
    P = C["P"]
    tf = transform_flops_per_apply(P["nx"], P["sub"])
    tach = tf / (t_pre * 1e-3) / 1e12
    roofs["precond_apply_fp64_alu"] = dict(
        bound="alu", achieved=round(tach, 2), peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
        frac=round(tach / FP64_VECTOR_PEAK_TFLOPS, 3), traffic=None,
        kernel="precond apply (passes A, B, C), FP64 transform arithmetic",
        flops_per_launch=round(tf), avg_ms=round(t_pre, 4),
        algorithmic_flops="per box, component and axis: pencils x n_axis^2/2 FMAs, forward and "
                          "inverse (even/odd butterfly), 2 flops per FMA")
    share = {"k_mupdate": pinfo["t_orth_update_ms"], "k_mdot": pinfo["t_orth_dot_ms"],
             "precond_apply": pinfo["t_precond_ms"], "k_curlcurl": pinfo["t_spmv_ms"]}
    dominant = max(share, key=share.get)
    pre_bytes = 16.0 * n_unk
    # a plain device copy of one vector, to calibrate HBM traffic counters
    cal = torch.empty_like(b)
    t_copy = time_events(lambda: cal.copy_(b), 10)
    del cal
    if args.ref_out:
        np.save(args.ref_out, x64.cpu().numpy())
    return {
        "metric": METRIC, "value": round(tts64, 2), "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(tts64, 2),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "256^3 Yee grid, PEC walls, 8^3 subdomains of 32^3 (overlap 1), "
                               "eps_r U[1,10] on 8^3 cubes, c=2, RHS N(0,1) seed 3; FGMRES(30) "
                               "FP64 to rel. residual 1e-8 with FlashMP RAS (FP64 transforms)",
                   "unknowns": n_unk, "solver": "fgmres(30)", "rtol": 1e-8},
        "iterations": info64["iterations"],
        "rel_residual_true": info64["rel_residual_true"],
        "precond_applies_per_s": round(1e3 / t_pre, 1),
        "precond_ms": round(t_pre, 4),
        "precond_plan": plan64,
        "precond_hbm_gbs_min_traffic": round(pre_bytes / (t_pre * 1e-3) / 1e9, 1),
        "spmv_ms": round(t_spmv, 4),
        "roofline": roofs[dominant],
        "roofline_all": roofs,
        "time_share_ms_per_solve": {k: round(v, 2) for k, v in share.items()},
        "copy_calibration": {"bytes": 16.0 * b.numel(), "avg_ms": round(t_copy, 4),
                             "GB/s": round(16.0 * b.numel() / (t_copy * 1e-3) / 1e9, 1)},
        "variants": {},
    }


def variant_leg(args):
    """FP32 or BF16 transforms on the 256^3 workload, error against the FP64 solution."""
    C = c3_context(args)
    torch, b = C["torch"], C["b"]
    hv, planv = C["tuned_handle"](args.prec)
    xv, infov, ttsv = C["run_solves"](hv, max(1, args.steps), args.warmup, args.prec)
    zv = hv.new_vector()
    tpv = C["time_events"](lambda: hv.apply_precond(b, zv), 10)
    out = dict(time_to_solution_ms=round(ttsv, 2), iterations=infov["iterations"],
               rel_residual_true=infov["rel_residual_true"],
               precond_applies_per_s=round(1e3 / tpv, 1), precond_ms=round(tpv, 4),
               precond_plan=planv)
    if args.ref_in:
        ref = torch.from_numpy(np.load(args.ref_in)).to(xv.device)
        out["rel_err_vs_fp64_solution"] = float(torch.linalg.vector_norm(xv - ref) /
                                                torch.linalg.vector_norm(ref))
    return out


def run_leg(args, emit=True):
    dev = "cuda:0"
    if args.leg == "main":
        res = main_leg(args)
    elif args.leg == "variant":
        res = variant_leg(args)
    elif args.leg == "batch":
        res = batch_leg(args, dev, log)
    elif args.leg == "learned":
        res = learned_leg(args, dev, log)
    elif args.leg == "convergence":
        res = convergence_leg(args, dev, log)
    elif args.leg == "cn":
        res = cn_leg(args, dev, log)
    elif args.leg == "whole":
        res = whole_leg(args, dev, log)
    elif args.leg == "c2":
        res = c2_leg(args, dev, log)
    else:
        raise SystemExit(f"unknown leg {args.leg}")
    if emit:
        print("LEG_RESULT " + json.dumps(res), flush=True)
    return res


def child(args, leg, extra=()):
    """Run one leg in a child process (each leg gets a fresh process), or in this
    process with --isolate 0; progress goes to stderr, the result comes back as
    JSON."""
    import subprocess
    opts = ["--steps", str(args.steps), "--warmup", str(args.warmup), "--config", args.config,
            "--pairs-rhs", str(args.pairs_rhs), "--pairs-per-rhs", str(args.pairs_per_rhs),
            "--epochs", str(args.epochs), "--graphs", str(args.graphs)] + list(extra)
    log(f"[bench] leg {leg} {' '.join(extra)}")
    if not args.isolate:
        sub = parse_args(["--leg", leg] + opts)
        t0 = time.perf_counter()
        res = run_leg(sub, emit=False)
        log(f"[bench] leg {leg} done in {time.perf_counter() - t0:.1f} s")
        return res
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--leg", leg] + opts
    p = subprocess.run(cmd, stdout=subprocess.PIPE, text=True)
    for line in p.stdout.splitlines():
        if line.startswith("LEG_RESULT "):
            return json.loads(line[len("LEG_RESULT "):])
    return dict(error=f"leg {leg} ended with status {p.returncode} and no result")


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--variants", default="fp32,bf16")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--learned", type=int, default=1, help="run the C5 learned-correction leg")
    ap.add_argument("--batch", type=int, default=1, help="run the 64-domain batch leg")
    ap.add_argument("--cn", type=int, default=1,
                    help="run the Crank-Nicolson time-stepping leg (256^3)")
    ap.add_argument("--convergence", type=int, default=1,
                    help="run the overlap / solver convergence study leg (128^3)")
    ap.add_argument("--pairs-rhs", type=int, default=100)
    ap.add_argument("--pairs-per-rhs", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--leg", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--prec", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--ref-out", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--ref-in", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--c2", type=int, default=1,
                    help="run the 128^3 leg (GPU solves compared with the CPU oracle's solve)")
    ap.add_argument("--c2-dir", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--graphs", type=int, default=1,
                    help="capture preconditioner applies in hipGraphs in every leg")
    ap.add_argument("--isolate", type=int, default=1,
                    help="1: every leg in a child process of its own; 0: all legs in this process")
    return ap.parse_args(argv)


def main():
    args = parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path; "
              "its kernels run one GPU's share of a sharded grid at its real shape",
              file=sys.stderr)
        sys.exit(2)
    if args.leg:
        run_leg(args)
        return

    # By default this process never touches the GPU: each leg runs in a child
    # process of its own and reports back, so one leg's failure is reported as
    # that leg's error instead of ending the whole run (--isolate 0 runs every
    # leg in this process, one after the other).
    import shutil
    import tempfile
    tmp = tempfile.mkdtemp(prefix="fmp_bench_")
    ref = os.path.join(tmp, "x64.npy")
    try:
        out = child(args, "main", ["--ref-out", ref])
        if "error" in out:
            print(json.dumps(dict(metric=METRIC, value=None, unit="ms", n_gpus=1, error=out["error"])),
                  flush=True)
            sys.exit(1)
        for prec in [v for v in args.variants.split(",") if v]:
            r = child(args, "variant", ["--prec", prec, "--ref-in", ref])
            if "time_to_solution_ms" in r:
                r["speedup_vs_fp64"] = round(out["value"] / r["time_to_solution_ms"], 3)
            out["variants"][prec] = r
        if args.batch:
            out["variants"]["batch_c4"] = child(args, "batch")
            out["variants"]["batch_c4_whole_domain_bf16"] = child(args, "whole")
            out["variants"]["batch_c4_whole_domain_fp32"] = child(args, "whole", ["--prec", "fp32"])
        if args.learned:
            out["variants"]["learned_c5"] = child(args, "learned")
        if args.convergence:
            out["variants"]["convergence_overlap"] = child(args, "convergence")
        if args.cn:
            out["variants"]["cn_time_stepping"] = child(args, "cn")
        if args.c2:
            c2dir = os.path.join(tmp, "c2")
            os.makedirs(c2dir, exist_ok=True)
            out["variants"]["c2"] = child(args, "c2", ["--c2-dir", c2dir])
        # CPU work only after every GPU leg, so it never competes with them
        if not args.no_cpu:
            from paper_2508_07193_amd import inputs
            out["cpu_baseline"] = cpu_baseline(inputs.make_problem(args.config), out["iterations"])
            if args.c2 and "runs" in out["variants"]["c2"]:
                log("[bench] CPU oracle: whole 128^3 BiCGSTAB solve")
                oc2, xo = cpu_oracle_c2()
                out["cpu_oracle_c2"] = oc2
                c2 = out["variants"]["c2"]
                xo = xo.ravel()
                for prec, r in c2["runs"].items():
                    f = os.path.join(c2dir, f"x_{prec}.npy")
                    if os.path.exists(f):
                        xg = np.load(f)
                        r["rel_err_vs_oracle_solution"] = float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))
                r64 = c2["runs"].get("fp64", {})
                if "time_to_solution_ms" in r64:
                    c2["speedup_vs_cpu_oracle"] = round(oc2["time_to_solution_s"] * 1e3 /
                                                        r64["time_to_solution_ms"], 1)
                log(f"[bench] CPU oracle 128^3: {oc2}")
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
