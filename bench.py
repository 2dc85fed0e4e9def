#!/usr/bin/env python
"""Benchmark: sgn(H) b applications per second on the 10^4 lattice.

Workload (one "step"): the 12 spin-colour point sources at the origin of a
10^4 lattice (synthetic SU(3) links, eps = 0.35, seed 10401, m0 = 1.6) at
mu = 0 (Lanczos) and mu = 0.2 (two-sided Lanczos): 24 sign applications in
one batched libnks call (outer basis, nested step, lift for every job).
k = 520 (mu = 0) and k = 620 (mu = 0.2) with ell = 64 are the smallest outer
sizes (in steps of 20) at which the oracle's own nested result is within
5e-9 of the converged sgn(A) b for every source, i.e. within the metric's
1e-8 with room for rounding (tests/golden/point12_10x4_sketch.npz).  The
full-vector error of every result is estimated on every run from the
references' Gaussian sketches, and measured exactly for four sources.

Prints ONE JSON line.  Extra sections: the mixed-precision path, the stencil
pass on a lattice far larger than the 256 MB last-level cache (its HBM
roofline), and the CPU oracle timed on a bounded sample.

Options: --gpus N (only 1), --steps K, --warmup W, --precision fp64|mixed,
--no-cpu, --no-large, --copy-calibration (time a plain copy kernel of
known size, for scaling hardware counters; prints its own JSON line).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "sgn(H)b applications/sec at 10^4, rel err 1e-8; stencil HBM GB/s vs peak"
DIMS = (10, 10, 10, 10)
EPS, LINK_SEED, M0 = 0.35, 10401, 1.6
MUS = (0.0, 0.2)
K_MU, ELL = {0.0: 520, 0.2: 620}, 64   # outer size per mu (Lanczos / two-sided), nested size
INFLIGHT = 1          # batches in flight on separate streams in the timed region
SERIAL_GROUPS = False    # --serial-groups
KERNEL_SOURCES = ("paper_0912_4457_amd/csrc/wilson.h", "paper_0912_4457_amd/csrc/outer.hip",
                  "paper_0912_4457_amd/csrc/nks_internal.h")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(paths=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def tuning_str(choice) -> str:
    return ",".join(f"{k}={int(v)}" for k, v in sorted(choice.items()))


def recorded_traffic(tuning=None):
    """Per-launch HBM bytes of the stencil pass from profiles/, if the kernel is
    unchanged and the counters were taken with the same launch tuning."""
    path = os.path.join(ROOT, "profiles", "stencil_point12_10x4_pmc.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k_, v_ = line.split(":", 1)
            vals[k_.strip()] = v_.strip()
    if vals.get("source_sha") != source_hash():
        return None
    # one counter set per launch tuning: "tuning" / "hbm_bytes_per_launch", then ".2", ".3", ...
    for suffix in ("", ".2", ".3", ".4"):
        if f"tuning{suffix}" not in vals and suffix:
            break
        if tuning is None or vals.get(f"tuning{suffix}") == tuning_str(tuning):
            try:
                return float(vals[f"hbm_bytes_per_launch{suffix}"])
            except (KeyError, ValueError):
                return None
    return None


def golden_samples():
    path = os.path.join(ROOT, "tests", "golden", "point12_10x4.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def make_jobs(nks, torch, ctx, precision, **policy):
    """The 24 jobs of the workload; policy keys (k, ell, tol, k_policy,
    ell_policy) override the fixed k = K_MU[mu], ell = ELL."""
    import nks_inputs as I
    links = I.su3_links(DIMS, EPS, LINK_SEED)
    lats, jobs = [], []
    for mu in MUS:
        lat = nks.Lattice(ctx, DIMS, links, m0=M0, mu=mu)
        lats.append(lat)
        for spin in range(4):
            for colour in range(3):
                b = torch.from_numpy(I.point_source(DIMS, spin, colour).ravel()).cuda()
                j = dict(lat=lat, b=b, k=K_MU[mu], ell=ELL, precision=precision, mu=mu, spin=spin,
                         colour=colour, x=torch.empty_like(b))
                j.update(policy)
                jobs.append(j)
    return lats, jobs


def errors_vs_golden(jobs, xs, gold):
    """Relative error of each result against the oracle's converged reference:
    the full-vector estimate from the reference's sketch for sign results
    (errors_vs_sketch), the error on the sampled entries of
    tests/golden/point12_10x4.json for overlap results (reference
    b + gamma5 sgn(A) b on the same entries)."""
    sk = errors_vs_sketch(jobs, xs, sketch_golden())
    sampled = sampled_errors(jobs, xs, gold)
    if sk is None:
        return sampled
    return [e if e is not None else (sampled[i] if sampled else None) for i, e in enumerate(sk)]


def sampled_errors(jobs, xs, gold):
    """Relative error on the sampled entries; for overlap jobs the reference is
    b + gamma5 sgn(A) b on the same entries."""
    import numpy as np
    if gold is None:
        return None
    errs = []
    for j, x in zip(jobs, xs):
        case = next(c for c in gold["cases"]
                    if c["mu"] == j["mu"] and c["spin"] == j["spin"] and c["colour"] == j["colour"])
        idx = np.asarray(case["idx"])
        ref = np.asarray(case["re"]) + 1j * np.asarray(case["im"])
        if j.get("overlap"):
            g5 = np.where((idx % 12) >= 6, -1.0, 1.0)
            ref = j["b"].cpu().numpy()[idx] + g5 * ref
        got = x.cpu().numpy()[idx]
        errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
    return errs


def full_golden():
    path = os.path.join(ROOT, "tests", "golden", "point4_full_10x4.npz")
    if not os.path.exists(path):
        return None
    import numpy as np
    return dict(np.load(path))


_SKETCH = {}


def sketch_golden():
    path = os.path.join(ROOT, "tests", "golden", "point12_10x4_sketch.npz")
    if not os.path.exists(path):
        return None
    import numpy as np
    return dict(np.load(path))


def errors_vs_sketch(jobs, xs, sk):
    """Full-vector relative errors of the plain sign results, estimated from
    the 256-row Gaussian sketch of each converged reference
    (tests/golden/point12_10x4_sketch.npz): |S x - S y| / (16 |y|), about 3 %
    relative spread.  None for overlap jobs (their reference is not sketched)."""
    import numpy as np
    import nks_inputs as I
    if sk is None:
        return None
    rows = int(sk["rows"])
    key = (xs[0].numel(), rows, int(sk["seed"]))
    if _SKETCH.get("key") != key:
        _SKETCH.update(key=key, S=I.sketch_rows(key[0], range(rows), key[2]))
    S = _SKETCH["S"]
    X = np.stack([x.cpu().numpy() for x in xs])
    SX = S @ X.T
    errs = []
    for i, j in enumerate(jobs):
        if j.get("overlap"):
            errs.append(None)
            continue
        c = [t for t in range(len(sk["mu"]))
             if sk["mu"][t] == j["mu"] and sk["spin"][t] == j["spin"] and sk["colour"][t] == j["colour"]][0]
        errs.append(float(np.linalg.norm(SX[:, i] - sk["sy"][c]) / (np.sqrt(rows) * sk["norm"][c])))
    return errs


def errors_vs_full(jobs, xs, full):
    """Full-vector relative errors for the sources with a complete reference
    (tests/golden/point4_full_10x4.npz): list of (mu, spin, colour, error)."""
    import numpy as np
    if full is None:
        return None
    out = []
    for i in range(len(full["mu"])):
        mu, spin, colour = float(full["mu"][i]), int(full["spin"][i]), int(full["colour"][i])
        for j, x in zip(jobs, xs):
            if j["mu"] == mu and j["spin"] == spin and j["colour"] == colour and not j.get("overlap"):
                ref = full["y"][i]
                got = x.cpu().numpy()
                out.append((mu, spin, colour, float(np.linalg.norm(got - ref) / np.linalg.norm(ref))))
    return out


def inflight_slots(nks, torch, jobs, n):
    """n independent copies of a batch (own outputs, workspace and stream), so
    that consecutive steps can be in flight together: while one batch runs
    its nested step (one workgroup per job) the next one's outer passes fill
    the rest of the GPU."""
    slots = []
    size = nks.workspace_size([(j["lat"], j["b"], j["x"], nks.make_opts(k=j["k"], ell=j["ell"],
                                                                          precision=j["precision"]))
                               for j in jobs])
    for i in range(n):
        js = jobs if i == 0 else [dict(j, x=torch.empty_like(j["b"])) for j in jobs]
        ws = torch.empty(size, dtype=torch.uint8, device="cuda")
        st = torch.cuda.Stream()
        slots.append((js, ws, st))
    return slots


def run_slots(nks, torch, slots, steps):
    for s in range(steps):
        js, ws, st = slots[s % len(slots)]
        with torch.cuda.stream(st):
            nks.sign_apply_batch(js, stats=False, workspace=ws)


def run_path(nks, torch, ctx, precision, steps, warmup, gold, profile, tune=True):
    lats, jobs = make_jobs(nks, torch, ctx, precision)
    tuned = None
    if tune:
        from paper_0912_4457_amd.autotune import autotune
        tuned = autotune(ctx, jobs, use_cache=False)
        log(f"[bench] autotune {precision}: {tuned['choice']} {tuned['timings']}")
        from paper_0912_4457_amd.autotune import schedule
        tuned["schedule"] = schedule(ctx, jobs)
        log(f"[bench] schedule {precision}: {tuned['schedule']['choice']} {tuned['schedule']['seconds_per_call']}")
    slots = inflight_slots(nks, torch, jobs, INFLIGHT)
    run_slots(nks, torch, slots, max(warmup, INFLIGHT))
    torch.cuda.synchronize()
    # timed region: the library's default path (graph replay, lattice groups
    # on concurrent streams), consecutive steps in flight on INFLIGHT streams
    t0 = time.perf_counter()
    run_slots(nks, torch, slots, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    one_dt = None
    if INFLIGHT > 1:
        t1 = time.perf_counter()
        run_slots(nks, torch, slots[:1], steps)
        torch.cuda.synchronize()
        one_dt = time.perf_counter() - t1
    prof = {}
    if profile:
        # per-kernel launch durations: the same steps again with the groups one
        # after another (overlapping groups would stretch every launch's span)
        # and HIP events on one launch in eight of each kernel class
        ctx.tune_set("concurrent_groups", 0)
        ctx.profile(True)
        for _ in range(steps):
            nks.sign_apply_batch(jobs, stats=False)
        torch.cuda.synchronize()
        for kc in ("stencil", "recurrence", "nested", "lift"):
            n, ms, by = ctx.profile_read(kc)
            prof[kc] = dict(launches=n, avg_ms=(ms / n if n else None), alg_bytes=(by / n if n else None))
        ctx.profile(False)
        ctx.tune_set("concurrent_groups", 0 if SERIAL_GROUPS else 1)
    xs, sts = nks.sign_apply_batch(jobs, stats=True)   # one more call for the per-job report
    torch.cuda.synchronize()
    errs = errors_vs_golden(jobs, xs, gold)
    full = errors_vs_full(jobs, xs, full_golden())
    # every in-flight copy computed the same results
    for js, _, _ in slots[1:]:
        for a, b in zip(jobs, js):
            if not torch.equal(a["x"], b["x"]):
                raise RuntimeError("in-flight copies of the batch disagree")
    return dict(seconds=dt, steps=steps, napps=len(jobs), prof=prof, stats=sts, errs=errs, tuned=tuned,
                one_stream_seconds=one_dt, full_errs=full)


def time_calls(nks, torch, jobs, steps, warmup, graph=True):
    """Seconds for `steps` batched calls (no stats, so graph mode replays)."""
    ctx = jobs[0]["lat"].ctx
    ctx.tune_set("graph", int(graph))
    for _ in range(warmup):
        nks.sign_apply_batch(jobs, stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        nks.sign_apply_batch(jobs, stats=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.tune_set("graph", 1)
    return dt


def policy_paths(nks, torch, ctx, gold, steps):
    """The same workload under the tolerance-driven policies: the plain
    ell-doubling / k-checkpoint rules and the learned network, FP64 at the
    workload's 1e-8 and mixed precision at 1e-6."""
    nks.load_policy(ctx)
    out = []
    for name, prec, pol, tol in (("fp64_doubling", "fp64", 1, 1e-8), ("fp64_learned", "fp64", 2, 1e-8),
                                 ("mixed_doubling", "mixed", 1, 1e-6), ("mixed_learned", "mixed", 2, 1e-6)):
        lats, jobs = make_jobs(nks, torch, ctx, prec, k=1400, ell=256, tol=tol, k_policy=pol, ell_policy=pol)
        dt = time_calls(nks, torch, jobs, steps, 1)
        xs, sts = nks.sign_apply_batch(jobs, stats=True)
        torch.cuda.synchronize()
        errs = errors_vs_golden(jobs, xs, gold)
        out.append({"path": name, "precision": prec, "tol": tol, "value": len(jobs) * steps / dt,
                    "ms_per_step": dt / steps * 1e3,
                    "max_rel_err_vs_oracle": max(errs) if errs else None,
                    "k_used_mean": sum(s["k_used"] for s in sts) / len(sts),
                    "ell_used": sorted(set(s["ell_used"] for s in sts)),
                    "status": sorted(set(s["status"] for s in sts))})
        log(f"[bench] {name}: {out[-1]['value']:.1f} app/s, err {out[-1]['max_rel_err_vs_oracle']}, "
            f"k mean {out[-1]['k_used_mean']:.0f}")
        for lat in lats:
            lat.close()
    return out


def overlap_path(nks, torch, ctx, gold, steps):
    """The overlap operator D_ov b = b + gamma5 sgn(A) b on the same 24 jobs."""
    lats, jobs = make_jobs(nks, torch, ctx, "fp64", overlap=True)
    dt = time_calls(nks, torch, jobs, steps, 1)
    xs, sts = nks.sign_apply_batch(jobs, stats=True)
    torch.cuda.synchronize()
    errs = errors_vs_golden(jobs, xs, gold)
    for lat in lats:
        lat.close()
    return {"value": len(jobs) * steps / dt, "unit": "overlap applications/s",
            "max_rel_err_vs_oracle": max(errs) if errs else None}


def multilevel_path(nks, torch, ctx, gold, steps):
    """Multi-level nesting (Sec. 4.5) on the same 24 jobs: ell = 64 -> 32 -> 16
    -> 8 -> 4 (RHi on a 4 x 4 matrix) against the one-level nested step, with
    the nested kernel's own device time (HIP events on every nested launch of
    4 calls, the lattice groups one after another)."""
    out = {}
    for name, deep in (("one_level", ()), ("five_levels", (32, 16, 8, 4))):
        lats, jobs = make_jobs(nks, torch, ctx, "fp64", ell_deep=deep)
        dt = time_calls(nks, torch, jobs, steps, 1)
        ctx.tune_set("concurrent_groups", 0)
        ctx.profile(True)
        for _ in range(4):
            nks.sign_apply_batch(jobs, stats=False)
        torch.cuda.synchronize()
        n, ms, _ = ctx.profile_read("nested")
        for kc in ("stencil", "recurrence", "lift"):      # release the other classes' events
            ctx.profile_read(kc)
        ctx.profile(False)
        ctx.tune_set("concurrent_groups", 0 if SERIAL_GROUPS else 1)
        xs, sts = nks.sign_apply_batch(jobs, stats=True)
        torch.cuda.synchronize()
        errs = errors_vs_golden(jobs, xs, gold)
        out[name] = {"ell": [ELL] + list(deep), "value": len(jobs) * steps / dt,
                     "nested_ms": ms / n if n else None,
                     "max_rel_err_vs_oracle": max(errs) if errs else None,
                     "levels_used": sorted(set(s["levels_used"] for s in sts)),
                     "rhi_iters": sorted(set(s["rhi_iters"] for s in sts))}
        log(f"[bench] {name}: {out[name]['value']:.1f} app/s, nested {out[name]['nested_ms']} ms, "
            f"err {out[name]['max_rel_err_vs_oracle']}")
        for lat in lats:
            lat.close()
    out["unit"] = "applications/s"
    return out


def workspace_bytes(nks, ctx, jobs):
    import ctypes
    opts = [nks.make_opts(k=j["k"], ell=j["ell"], double_pass=j.get("double_pass", False)) for j in jobs]
    arr = (nks.Job * len(jobs))()
    for i, (j, o) in enumerate(zip(jobs, opts)):
        arr[i].lat, arr[i].b, arr[i].x = j["lat"].h.value, j["b"].data_ptr(), j["x"].data_ptr()
        arr[i].opts = ctypes.pointer(o)
    sz = ctypes.c_size_t()
    ctx.check(nks.lib().nks_workspace_size(ctx.h, len(jobs), arr, ctypes.byref(sz)))
    return sz.value


def double_pass_path(nks, torch, ctx, gold, steps, large=True):
    """Double-pass mode (Sec. 4.4): the same 24 jobs (results identical to the
    single-pass ones bit for bit), and 24 point sources on a 24^4 lattice,
    whose single-pass basis store at k = 500 would not fit in HBM."""
    import numpy as np
    lats, jobs = make_jobs(nks, torch, ctx, "fp64", double_pass=True)
    dt = time_calls(nks, torch, jobs, steps, 1)
    xs, sts = nks.sign_apply_batch(jobs, stats=True)
    torch.cuda.synchronize()
    errs = errors_vs_golden(jobs, xs, gold)
    out = {"value": len(jobs) * steps / dt, "unit": "applications/s",
           "max_rel_err_vs_oracle": max(errs) if errs else None,
           "workspace_GB": workspace_bytes(nks, ctx, jobs) / 1e9,
           "single_pass_workspace_GB": workspace_bytes(nks, ctx, [dict(j, double_pass=False) for j in jobs]) / 1e9}
    for lat in lats:
        lat.close()
    log(f"[bench] double pass 10^4: {out['value']:.1f} app/s, err {out['max_rel_err_vs_oracle']}, "
        f"workspace {out['workspace_GB']:.2f} GB (single pass {out['single_pass_workspace_GB']:.1f} GB)")
    if not large:
        return out
    import nks_inputs as I
    dims = (24, 24, 24, 24)
    links = I.su3_links(dims, EPS, LINK_SEED)
    big = []
    blats = []
    for mu in MUS:
        lat = nks.Lattice(ctx, dims, links, m0=M0, mu=mu)
        blats.append(lat)
        for spin in range(4):
            for colour in range(3):
                b = torch.from_numpy(I.point_source(dims, spin, colour).ravel()).cuda()
                big.append(dict(lat=lat, b=b, x=torch.empty_like(b), k=K_MU[mu], ell=ELL, double_pass=True, mu=mu))
    nks.sign_apply_batch(big, stats=False)                 # warm (graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, _ = nks.sign_apply_batch(big, stats=False)
    torch.cuda.synchronize()
    dtb = time.perf_counter() - t0
    # accuracy by the sgn^2 estimate of Sec. 3 on one source per mu
    est = []
    for idx in (0, len(big) // 2):
        j = big[idx]
        x2, _ = nks.sign_apply(j["lat"], xs[idx], k=j["k"], ell=ELL, double_pass=True, stats=False)
        torch.cuda.synchronize()
        est.append(float(torch.linalg.vector_norm(x2 - j["b"]) / (2 * torch.linalg.vector_norm(j["b"]))))
    out["large"] = {"lattice": "24^4", "jobs": len(big), "k": {str(m): k for m, k in K_MU.items()}, "ell": ELL, "value": len(big) / dtb,
                    "seconds_per_call": dtb, "workspace_GB": workspace_bytes(nks, ctx, big) / 1e9,
                    "single_pass_workspace_GB": workspace_bytes(nks, ctx, [dict(j, double_pass=False)
                                                                          for j in big]) / 1e9,
                    "sgn2_error_estimate": est}
    log(f"[bench] double pass 24^4: {out['large']['value']:.2f} app/s, sgn^2 estimate {est}, "
        f"workspace {out['large']['workspace_GB']:.1f} GB (single pass {out['large']['single_pass_workspace_GB']:.0f} GB)")
    for lat in blats:
        lat.close()
    return out


def deflation_path(nks, torch, ctx, gold, steps, m=16):
    """Deflation (App. C steps 1 and 6) with eigenpairs from the GPU
    eigensolver, on the 12 point sources of the workload at each mu (left
    eigenvectors from A(-mu) when mu != 0): the eigensolve, then plain and
    deflated batches at k = 500, 300 and 200 (ell = 64) with their errors
    against the golden references."""
    import nks_inputs as I
    links = I.su3_links(DIMS, EPS, LINK_SEED)
    out = {"eigenpairs": m, "unit": "applications/s", "eigensolves": [], "runs": []}
    for mu in MUS:
        lat = nks.Lattice(ctx, DIMS, links, m0=M0, mu=mu)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, res, it = lat.compute_deflation(m, tol=1e-10)
        t_eig = time.perf_counter() - t0
        out["eigensolves"].append({"mu": mu, "seconds": t_eig, "iterations": it, "max_residual": float(res.max()),
                                   "abs_lambda_range": [float(abs(lam).min()), float(abs(lam).max())],
                                   "max_abs_imag_lambda": float(abs(lam.imag).max())})
        log(f"[bench] eigensolve mu={mu} {m} pairs: {t_eig:.2f} s, {it} iterations, residual {res.max():.1e}")
        base = []
        for spin in range(4):
            for colour in range(3):
                b = torch.from_numpy(I.point_source(DIMS, spin, colour).ravel()).cuda()
                base.append(dict(lat=lat, b=b, x=torch.empty_like(b), ell=ELL, precision="fp64", mu=mu,
                                 spin=spin, colour=colour))
        for k in (500, 300, 200):
            for defl in (False, True):
                jobs = [dict(j, k=k, deflate=defl) for j in base]
                dt = time_calls(nks, torch, jobs, steps, 1)
                xs, _ = nks.sign_apply_batch(jobs, stats=True)
                torch.cuda.synchronize()
                errs = errors_vs_golden(jobs, xs, gold)
                out["runs"].append({"mu": mu, "k": k, "deflated": defl, "value": len(jobs) * steps / dt,
                                    "max_rel_err_vs_oracle": max(errs) if errs else None})
                log(f"[bench] deflation mu={mu} k={k} deflated={defl}: {out['runs'][-1]['value']:.1f} app/s, "
                    f"err {out['runs'][-1]['max_rel_err_vs_oracle']}")
        lat.close()
    return out


def c2_path(nks, torch, ctx):
    """The two-sided 8^4 workload (eps = 0.4, mu = 0.3, Gaussian source,
    k = 800, ell = 150), FP64 and mixed, plain and deflated by the GPU
    eigensolver's 16 pairs, each result's error against the oracle's converged
    reference (tests/golden/c2_8x4.npz), and the plain FP64 result at the
    oracle's p against the oracle's own run at the same (k, ell, p)."""
    import numpy as np
    import nks_inputs as I
    path = os.path.join(ROOT, "tests", "golden", "c2_8x4.npz")
    if not os.path.exists(path):
        return None
    g = dict(np.load(path))
    if "m" not in g or "y_run" not in g:
        return None
    dims = (8, 8, 8, 8)
    lat = nks.Lattice(ctx, dims, I.su3_links(dims, 0.4, 8401), m0=M0, mu=0.3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, res, it = lat.compute_deflation(int(g["m"]), tol=1e-10)
    t_eig = time.perf_counter() - t0
    b = torch.from_numpy(I.gaussian_source(dims, 8402).ravel()).cuda()
    ref = g["y_ref"]
    k, ell = int(g["k_run"]), int(g["ell_run"])
    out = {"workload": f"8^4, eps=0.4, mu=0.3, Gaussian source, k={k}, ell={ell}, {int(g['m'])} deflated eigenpairs",
           "eigensolve_seconds": t_eig, "eigensolve_iterations": it, "max_residual": float(res.max()),
           "oracle_err_same_k_deflated": float(g["oracle_err_deflated"]),
           "oracle_err_same_k_plain": float(g["oracle_err_run"]),
           "reference_change_from_k_check": float(g["change_from_k_check"]), "results": []}
    for prec in ("fp64", "mixed"):
        for defl in (True, False):
            nks.sign_apply(lat, b, k=k, ell=ell, deflate=defl, precision=prec)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, st = nks.sign_apply(lat, b, k=k, ell=ell, deflate=defl, precision=prec)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            err = float(np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref))
            out["results"].append({"precision": prec, "deflated": defl, "rel_err_vs_converged": err,
                                   "seconds": dt, "status": st["status"]})
            log(f"[bench] C2 {prec} deflated={defl}: rel err {err:.2e} vs converged, {dt * 1e3:.1f} ms")
    x, _ = nks.sign_apply(lat, b, k=k, ell=ell, p=float(g["p_run"]))
    y = g["y_run"]
    out["fp64_plain_vs_oracle_same_k_ell_p"] = float(np.linalg.norm(x.cpu().numpy() - y) / np.linalg.norm(y))
    out["oracle_rounding_response_same_k_ell_p"] = float(g["run_rounding_response"])
    lat.close()
    return out


def uneven_sketch():
    path = os.path.join(ROOT, "tests", "golden", "uneven64_sketch.npz")
    if not os.path.exists(path):
        return None
    import numpy as np
    return dict(np.load(path))


def uneven_errors(jobs, xs, sk):
    """Per-job full-vector errors of the uneven batch from the sketched
    references, with how many exceed their job's tolerance."""
    import numpy as np
    import nks_inputs as I
    if sk is None:
        return {}
    rows, seed = int(sk["rows"]), int(sk["seed"])
    errs = []
    for i, (j, x) in enumerate(zip(jobs, xs)):
        n = x.numel()
        if _SKETCH.get(("uneven", n)) is None:
            _SKETCH[("uneven", n)] = I.sketch_rows(n, range(rows), seed)
        sx = _SKETCH[("uneven", n)] @ x.cpu().numpy()
        errs.append(float(np.linalg.norm(sx - sk["sy"][i]) / (np.sqrt(rows) * sk["norm"][i])))
    tols = [j["tol"] for j in jobs]
    assert np.allclose(tols, sk["tol"]), "job list differs from the sketched references"
    above = [i for i, (e, t) in enumerate(zip(errs, tols)) if e > t]
    return {"rel_err_per_job": errs, "jobs_above_tolerance": above,
            "error_summary": {f"tol {t:g}": max(e for e, tt in zip(errs, tols) if tt == t) for t in sorted(set(tols))}}


def uneven_batch(nks, torch, ctx, steps):
    """64 point sources over nine lattices (6^4, 8^4, 10^4 x mu in {0, 0.1,
    0.3}) with tolerances 1e-6 / 1e-8, in one batched call: plain policies
    eager and graph-replayed, and the learned policy graph-replayed."""
    import numpy as np
    import nks_inputs as I
    rng = np.random.default_rng(64)
    lats = []
    for dims, seed in (((6, 6, 6, 6), 6601), ((8, 8, 8, 8), 8801), ((10, 10, 10, 10), 10401)):
        u = I.su3_links(dims, EPS, seed)
        for mu in (0.0, 0.1, 0.3):
            lats.append(nks.Lattice(ctx, dims, u, m0=M0, mu=mu))
    base = []
    for i in range(64):
        lat = lats[i % len(lats)]
        b = torch.from_numpy(I.point_source(lat.dims, int(rng.integers(4)), int(rng.integers(3)),
                                            int(rng.integers(lat.V))).ravel()).cuda()
        base.append(dict(lat=lat, b=b, x=torch.empty_like(b), k=1400, ell=256,
                         tol=float(rng.choice([1e-6, 1e-8])), precision="fp64"))
    res = {"jobs": 64, "lattices": "6^4, 8^4, 10^4 x mu in {0, 0.1, 0.3}", "tolerances": [1e-6, 1e-8],
           "rel_err_how": "full-vector relative error of each job against the oracle's converged reference, "
                          "estimated from its 256-row Gaussian sketch (tests/golden/uneven64_sketch.npz)"}
    sk = uneven_sketch()
    nks.load_policy(ctx)
    for name, pol, graph in (("doubling_eager", 1, False), ("doubling_graph", 1, True), ("learned_graph", 2, True)):
        jobs = [dict(j, k_policy=pol, ell_policy=pol) for j in base]
        dt = time_calls(nks, torch, jobs, steps, 1, graph=graph)
        res[name] = {"value": 64 * steps / dt, "ms_per_call": dt / steps * 1e3}
        res[name].update(uneven_errors(jobs, [j["x"] for j in jobs], sk))
        log(f"[bench] uneven batch {name}: {res[name]['value']:.1f} app/s, errors {res[name].get('error_summary')}")
    # the same 64 jobs one at a time (single calls in sequence, doubling
    # policies, eager: a captured graph pays off only when the same call
    # repeats, and 64 different calls would only churn the graph cache):
    # what the batch saves
    jobs = [dict(j, k_policy=1, ell_policy=1) for j in base]
    ctx.tune_set("graph", 0)
    for j in jobs:
        nks.sign_apply(j["lat"], j["b"], k=j["k"], ell=j["ell"], tol=j["tol"], stats=False, out=j["x"],
                       k_policy=1, ell_policy=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for j in jobs:
            nks.sign_apply(j["lat"], j["b"], k=j["k"], ell=j["ell"], tol=j["tol"], stats=False, out=j["x"],
                           k_policy=1, ell_policy=1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.tune_set("graph", 1)
    res["doubling_one_at_a_time"] = {"value": 64 * steps / dt, "ms_per_call": dt / steps * 1e3, "graph": False}
    res["doubling_one_at_a_time"].update(uneven_errors(jobs, [j["x"] for j in jobs], sk))
    log(f"[bench] uneven batch one at a time: {res['doubling_one_at_a_time']['value']:.1f} app/s")
    for lat in lats:
        lat.close()
    return res


def stencil_large(nks, torch, ctx, precision):
    """Stencil pass on a 32^4 lattice (one source, 0.4-0.8 GB per pass): HBM-bound."""
    import numpy as np
    dims = (32, 32, 32, 32)
    V = int(np.prod(dims))
    rng = np.random.default_rng(1)
    # links: random SU(3)-like unitary matrices are not needed for timing; use
    # the identity plus noise re-unitarised cheaply on the GPU side is overkill,
    # so take unit links (the stencil does the same work for any link values)
    links = torch.zeros((V, 4, 3, 3), dtype=torch.complex128)
    links[..., 0, 0] = links[..., 1, 1] = links[..., 2, 2] = 1
    lat = nks.Lattice(ctx, dims, links.cuda(), m0=M0, mu=0.0)
    b = torch.from_numpy(rng.standard_normal(12 * V) + 1j * rng.standard_normal(12 * V)).cuda()
    nks.outer_basis(lat, b, 4, precision=precision)   # warm
    ctx.profile(True)
    nks.outer_basis(lat, b, 16, precision=precision)
    n, ms, by = ctx.profile_read("stencil")
    ctx.profile_read("recurrence")
    ctx.profile(False)
    lat.close()
    torch.cuda.synchronize()
    achieved = by / (ms * 1e-3) / 1e9
    return {"lattice": "32^4", "sources": 1, "precision": precision, "timed_launches": n,
            "avg_ms": ms / n, "alg_bytes_per_launch": by / n, "achieved_GBps": achieved,
            "peak_GBps": HBM_PEAK_GBPS, "frac": achieved / HBM_PEAK_GBPS}


_CPU_OPS = {}


def _cpu_init(barrier):
    """Worker of the CPU baseline: single-threaded BLAS, the workload's operators."""
    for v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    import nks_inputs as I
    from oracle import dirac
    links = I.su3_links(DIMS, EPS, LINK_SEED)
    for mu in MUS:
        _CPU_OPS[mu] = dirac.Operator(links, DIMS, M0, mu)
    barrier.wait()


def _cpu_job(job):
    import nks_inputs as I
    from oracle import nested
    mu, spin, colour = job
    t0 = time.perf_counter()
    nested.sign_apply(_CPU_OPS[mu], I.point_source(DIMS, spin, colour), K_MU[mu], ELL)
    return time.perf_counter() - t0


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The oracle's nested method on the whole workload (the 24 jobs of one
    step, k = K_MU[mu], ell = ELL), one single-threaded process per host core (at
    most 16), jobs handed out as workers become free; the timer starts once
    every worker has built its operators.  Also the single-core rate from a
    2-job sample in this process."""
    import multiprocessing as mp
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    nproc = min(16, avail)
    jobs = [(mu, s, c) for mu in MUS for s in range(4) for c in range(3)]
    ctxm = mp.get_context("spawn")
    barrier = ctxm.Barrier(nproc + 1)
    saved = {v: os.environ.get(v) for v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS")}
    for v in saved:
        os.environ[v] = "1"                       # inherited by the spawned workers
    try:
        with ctxm.Pool(nproc, initializer=_cpu_init, initargs=(barrier,)) as pool:
            barrier.wait()
            t0 = time.perf_counter()
            per_job = pool.map(_cpu_job, jobs, chunksize=1)
            dt = time.perf_counter() - t0
    finally:
        for v, old in saved.items():
            if old is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = old
    # single core, in this process (BLAS limited to one thread)
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    _cpu_init(type("NoBarrier", (), {"wait": staticmethod(lambda: None)})())
    sample = [(0.0, 0, 0), (0.2, 0, 0)]
    t1 = time.perf_counter()
    for j in sample:
        _cpu_job(j)
    dt1 = time.perf_counter() - t1
    return {"value": len(jobs) / dt, "unit": "applications/s", "cores": nproc, "kind": "oracle",
            "sample": f"all {len(jobs)} jobs of one step (12 point sources at mu = 0 and 0.2 on the 10^4 "
                      f"lattice, nested method k={K_MU[0.0]} / {K_MU[0.2]} ell={ELL}, scipy CSR + LAPACK), one single-threaded "
                      f"process per core on {nproc} of {avail} available cores: {dt:.1f} s "
                      f"(job times {min(per_job):.1f}-{max(per_job):.1f} s)",
            "nproc": os.cpu_count(), "cores_available": avail, "cpu_model": _cpu_model(), "blas_threads": 1,
            "single_core": {"value": len(sample) / dt1, "unit": "applications/s", "cores": 1,
                            "sample": f"2 jobs (point source (0,0) at mu = 0 and mu = 0.2), one thread: "
                                      f"{dt1:.1f} s"}}


def copy_calibration(torch):
    n = 1 << 28   # 2 GiB of float64 read, 2 GiB written
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y.copy_(x)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"copy_calibration": True, "bytes_read": 8 * n, "bytes_written": 8 * n,
                      "seconds": dt, "GBps": 16 * n / dt / 1e9}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the policy and uneven-batch sections")
    ap.add_argument("--serial-groups", action="store_true",
                    help="run the lattice groups one after another everywhere (for kernel traces whose "
                         "per-launch durations must not include overlap)")
    ap.add_argument("--probe", action="store_true",
                    help="short run of the main path only (for hardware-counter passes)")
    ap.add_argument("--tune", default="", help="launch tuning for --probe, e.g. xcd_map=3,split_dual=1,min_waves=1")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}): jobs are independent "
              f"sign applications; sharding sources over GPUs is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if a.copy_calibration:
        copy_calibration(torch)
        return
    import paper_0912_4457_amd as nks
    ctx = nks.Context(0)
    if a.serial_groups:
        global SERIAL_GROUPS
        SERIAL_GROUPS = True
        ctx.tune_set("concurrent_groups", 0)
    gold = golden_samples()

    if a.probe:
        for kv in filter(None, a.tune.split(",")):
            k_, v_ = kv.split("=")
            ctx.tune_set(k_.strip(), int(v_))
        lats, jobs = make_jobs(nks, torch, ctx, a.precision)
        for _ in range(max(1, a.steps)):
            nks.sign_apply_batch(jobs, stats=False)
        torch.cuda.synchronize()
        print(json.dumps({"probe": True, "precision": a.precision, "calls": max(1, a.steps), "tune": a.tune}))
        return
    log(f"[bench] {a.precision} path: 24 jobs per step, {a.warmup} warmup + {a.steps} timed steps")
    main_run = run_path(nks, torch, ctx, a.precision, a.steps, a.warmup, gold, profile=True)
    other = "mixed" if a.precision == "fp64" else "fp64"
    log(f"[bench] {other} path for comparison")
    other_run = run_path(nks, torch, ctx, other, max(2, a.steps // 2), 1, gold, profile=False)
    if main_run["tuned"]:                       # the comparison path re-tuned the context
        for k_, v_ in {**main_run["tuned"]["choice"], **main_run["tuned"]["schedule"]["choice"]}.items():
            ctx.tune_set(k_, v_)
    lats_g, jobs_g = make_jobs(nks, torch, ctx, a.precision)
    graph_dt = time_calls(nks, torch, jobs_g, a.steps, 1, graph=True)
    eager_dt = time_calls(nks, torch, jobs_g, a.steps, 1, graph=False)
    ctx.tune_set("pipeline_groups", 1)
    pipe_dt = time_calls(nks, torch, jobs_g, a.steps, 1, graph=True)
    ctx.tune_set("pipeline_groups", 0)
    ctx.tune_set("concurrent_groups", 0)
    serial_dt = time_calls(nks, torch, jobs_g, a.steps, 1, graph=True)
    ctx.tune_set("concurrent_groups", 0 if SERIAL_GROUPS else 1)
    for lat in lats_g:
        lat.close()
    paths = uneven = overlap_res = multilevel = double_pass = deflation = c2 = None
    if not a.no_extra:
        log("[bench] policy paths")
        paths = policy_paths(nks, torch, ctx, gold, max(2, a.steps // 2))
        log("[bench] overlap operator")
        overlap_res = overlap_path(nks, torch, ctx, gold, a.steps)
        log("[bench] multi-level nesting")
        multilevel = multilevel_path(nks, torch, ctx, gold, a.steps)
        log("[bench] deflation with GPU eigenpairs")
        deflation = deflation_path(nks, torch, ctx, gold, a.steps)
        log("[bench] double-pass mode")
        double_pass = double_pass_path(nks, torch, ctx, gold, a.steps, large=not a.no_large)
        log("[bench] uneven batch")
        uneven = uneven_batch(nks, torch, ctx, 2)
        log("[bench] 8^4 two-sided workload (C2)")
        c2 = c2_path(nks, torch, ctx)
    large = None
    if not a.no_large:
        log("[bench] stencil pass on a 32^4 lattice")
        large = stencil_large(nks, torch, ctx, "fp64")
    cpu = None
    if not a.no_cpu:
        log("[bench] CPU oracle sample")
        cpu = cpu_baseline()

    dt = main_run["seconds"]
    value = main_run["napps"] * a.steps / dt
    st = main_run["prof"]["stencil"]
    achieved = st["alg_bytes"] / (st["avg_ms"] * 1e-3) / 1e9
    traffic = recorded_traffic(main_run["tuned"]["choice"] if main_run["tuned"] else None)
    sts = main_run["stats"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "applications/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32 basis + f64 scalars",
        "data": "synthetic (seeded SU(3) links and point sources)",
        "config": {"workload": "point12_10x4: 10^4 lattice, 12 point sources x mu in {0, 0.2}, "
                               f"eps=0.35, m0=1.6, k={K_MU[0.0]} (mu = 0) / {K_MU[0.2]} (mu = 0.2), ell={ELL}",
                   "applications_per_step": main_run["napps"], "k": {str(m): k for m, k in K_MU.items()},
                   "ell": ELL,
                   "batches_in_flight": INFLIGHT},
        "roofline": {"bound": "hbm", "kernel": "outer stencil pass (A v fused with the recurrence terms)",
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "alg_bytes_per_launch": st["alg_bytes"], "avg_launch_ms": st["avg_ms"],
                     "timed_launches": st["launches"],
                     "launch_timing": "HIP events on the launch stream, one launch in eight, over a second pass "
                                      "of the timed steps with the lattice groups one after another"},
        "cpu_baseline": cpu,
        "kernels": main_run["prof"],
        "max_rel_err_vs_oracle": (max(main_run["errs"]) if main_run["errs"] else None),
        "rel_err_vs_oracle_per_source": main_run["errs"],
        "rel_err_vs_oracle_how": "full-vector relative error of each of the 24 results against the oracle's "
                                 "converged reference, estimated from a 256-row seeded Gaussian sketch of the "
                                 "reference (tests/golden/point12_10x4_sketch.npz; about 3 % relative spread); "
                                 "full_vector_rel_err: exact, complete vectors of 4 sources "
                                 "(tests/golden/point4_full_10x4.npz)",
        "full_vector_rel_err": ([{"mu": m, "spin": sp, "colour": co, "rel_err": e}
                                 for m, sp, co, e in main_run["full_errs"]] if main_run["full_errs"] else None),
        "other_path_full_vector_rel_err": ([{"mu": m, "spin": sp, "colour": co, "rel_err": e}
                                            for m, sp, co, e in other_run["full_errs"]]
                                           if other_run["full_errs"] else None),
        "k_used": [s["k_used"] for s in sts],
        "ell_used": sorted(set(s["ell_used"] for s in sts)),
        "p_used": sorted(set(round(s["p_used"], 4) for s in sts)),
        "other_path": {"precision": other,
                       "value": other_run["napps"] * other_run["steps"] / other_run["seconds"],
                       "max_rel_err_vs_oracle": (max(other_run["errs"]) if other_run["errs"] else None),
                       "rel_err_vs_oracle_per_source": other_run["errs"]},
        "batches_in_flight": {"count": INFLIGHT, "value": value,
                              "one_batch_at_a_time_value": (main_run["napps"] * a.steps / main_run["one_stream_seconds"]
                                                            if main_run["one_stream_seconds"] else None)},
        "graph_replay": {"value": main_run["napps"] * a.steps / graph_dt,
                         "eager_value": main_run["napps"] * a.steps / eager_dt,
                         "groups_one_after_another_value": main_run["napps"] * a.steps / serial_dt,
                         "pipelined_groups_value": main_run["napps"] * a.steps / pipe_dt},
        "policy_paths": paths,
        "overlap": overlap_res,
        "multilevel": multilevel,
        "double_pass": double_pass,
        "deflation": deflation,
        "uneven_batch": uneven,
        "c2_8x4": c2,
        "stencil_large": large,
        "tuning": main_run["tuned"],
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
