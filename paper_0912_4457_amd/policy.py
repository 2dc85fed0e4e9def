"""Learned ell/k policy (not part of the paper): training targets from label
runs, training on the library's own network kernels, and the network file.

The method needs an outer size k and an inner size ell.  The plain policies
(NKS_POLICY_DOUBLING) find them by checkpoints: k every 100 outer steps
until the weighted coefficient change is <= tol/4, ell by doubling from 16
until the change is <= tol/10.  The learned policy predicts both from
features of the probe Ritz matrix H_100 and verifies the prediction once
(see nks_policy_load in the public header).

Training data come from ``nks_policy_label`` runs on seeded synthetic
lattices: for every job the weighted error e_i of the nested result at
k_i = 20 (i + 1) against the job's full-length result, and the ell-doubling
changes at each k_i.  For a tolerance tau:

* k* = (first k_i from which every later e_i stays <= tau/4) + 40, the size
  whose verification against k* - 40 passes;
* ell* = the inner size 16 * 2^s of the first doubling step s at k* whose
  change is <= tau/10 (256 if none).

The network (16 -> 64 -> 64 -> 2, SiLU) regresses (log10 k*, log10 ell*)
from the normalised features; it is trained with nks_mlp_backward and
nks_mlp_adam_step on the GPU.  After training the outputs are shifted
against the asymmetric costs of a wrong guess: k up by the 85th percentile
of the held-out under-prediction (a short k costs a fall-back to the
checkpoints, a long one only extra outer steps), ell down to the 10th
percentile (a small start costs one more doubling at small size, a large
one a dense Roberts-Higham step eight times dearer per doubling).

    python -m paper_0912_4457_amd.policy --out policy_net.json --lattices 120
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

NFEAT = 16
NPARAMS = 5378
NFLOATS = NPARAMS + 2 * NFEAT + 4
LABEL_NK, LABEL_NELL, LABEL_DK = 60, 4, 20
LABEL_WORDS = NFEAT + LABEL_NK * (1 + LABEL_NELL)
ELL0 = 16
VERIFY_DK = 40
TOLS = (1e-6, 1e-7, 1e-8, 1e-9, 1e-10)
REF_MARGIN = 100           # k* must lie this far below the reference length
DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "policy_net.json")
SIZES = ((16, 64), (64, 64), (64, 2))


# ------------------------------------------------------------------ targets
def targets(label, tol: float, k_ref: int):
    """(features, (log10 k*, log10 ell*)) of one label row at tolerance tol,
    or None when the row does not resolve tol below k_ref - REF_MARGIN."""
    label = np.asarray(label, dtype=np.float64)
    if label.shape != (LABEL_WORDS,) or not np.all(np.isfinite(label[:NFEAT])):
        return None
    f = label[:NFEAT].copy()
    f[6] = math.log10(tol)
    e = label[NFEAT:NFEAT + LABEL_NK]
    trace = label[NFEAT + LABEL_NK:].reshape(LABEL_NK, LABEL_NELL)
    ks = LABEL_DK * (np.arange(LABEL_NK) + 1)
    valid = np.isfinite(e) & (ks <= k_ref)
    if not valid.any():
        return None
    last = int(np.nonzero(valid)[0][-1])
    good = valid & (e <= tol / 4)
    # first index from which every later valid entry stays good
    i_acc = None
    for i in range(last, -1, -1):
        if not valid[i]:
            continue
        if good[i]:
            i_acc = i
        else:
            break
    if i_acc is None:
        return None
    kstar = int(ks[i_acc]) + VERIFY_DK
    if kstar > k_ref - REF_MARGIN:
        return None
    tr = trace[kstar // LABEL_DK - 1]
    ell = ELL0 * 2 ** LABEL_NELL
    for s in range(LABEL_NELL):
        if np.isfinite(tr[s]) and tr[s] <= tol / 10:
            ell = ELL0 * 2 ** s
            break
    return f, (math.log10(kstar), math.log10(ell))


def dataset(labels, k_refs, groups, tols=TOLS):
    """Stack targets of many label rows: X (n, 16), T (n, 2), group id (n)."""
    X, T, G = [], [], []
    for row, kr, g in zip(labels, k_refs, groups):
        for tol in tols:
            r = targets(row, tol, kr)
            if r is not None:
                X.append(r[0])
                T.append(r[1])
                G.append(g)
    return np.asarray(X, np.float64).reshape(-1, NFEAT), np.asarray(T, np.float64).reshape(-1, 2), np.asarray(G)


# ------------------------------------------------------------------ network file
def normalisation(X, T):
    fm, fs = X.mean(axis=0), X.std(axis=0)
    const = fs < 1e-6
    fm[const], fs[const] = 0.0, 1.0          # constant features pass through (f0 = 1 acts as a bias)
    tm, ts = T.mean(axis=0), T.std(axis=0)
    ts[ts < 1e-6] = 1.0
    return fm, fs, tm, ts


def init_params(seed: int = 0):
    """Glorot-normal weights, zero biases, flattened in the kernel order
    W1[16][64], b1, W2[64][64], b2, W3[64][2], b3."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in SIZES:
        parts.append((rng.standard_normal((a, b)) * math.sqrt(2.0 / (a + b))).ravel())
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)


def pack(params, fm, fs, tm, ts):
    blob = np.concatenate([np.asarray(params, np.float32).ravel(), fm, fs, tm, ts]).astype(np.float32)
    assert blob.size == NFLOATS
    return blob


def save(path, blob, meta):
    blob = np.asarray(blob, np.float32)
    with open(path, "w") as fh:
        json.dump({"format": "nks-policy-1", "nfloats": int(blob.size), "blob": [float(v) for v in blob],
                   "meta": meta}, fh, indent=1)


def load(path=DEFAULT_PATH):
    with open(path) as fh:
        d = json.load(fh)
    if d.get("format") != "nks-policy-1" or d.get("nfloats") != NFLOATS:
        raise ValueError(f"{path}: not a policy network file of {NFLOATS} floats")
    return np.asarray(d["blob"], np.float32), d.get("meta", {})


# ------------------------------------------------------------------ training (GPU kernels)
def train(ctx, Xn, Tn, steps: int = 4000, lr: float = 3e-3, seed: int = 0, log=None):
    """Adam on 0.5 * mean ||net(Xn) - Tn||^2, full batch, cosine learning rate.
    Every forward, backward and update runs in libnks."""
    import torch
    from . import mlp_adam_step, mlp_backward
    P = torch.from_numpy(init_params(seed)).cuda()
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    Xd = torch.from_numpy(np.ascontiguousarray(Xn, np.float32)).cuda()
    Td = torch.from_numpy(np.ascontiguousarray(Tn, np.float32)).cuda()
    hist = []
    for t in range(1, steps + 1):
        loss, g = mlp_backward(ctx, P, Xd, Td)
        a = lr * 0.5 * (1.0 + math.cos(math.pi * (t - 1) / steps))
        mlp_adam_step(ctx, P, g, M, V, t, max(a, lr * 0.01))
        if t == 1 or t % 500 == 0 or t == steps:
            hist.append((t, float(loss.cpu())))
            if log:
                log(f"[policy] step {t} loss {hist[-1][1]:.5f}")
    return P.cpu().numpy(), hist


def predict(ctx, params, fm, fs, tm, ts, X):
    from . import mlp_forward
    Xn = ((X - fm) / fs).astype(np.float32)
    y = mlp_forward(ctx, params, Xn).cpu().numpy().astype(np.float64)
    return y * ts + tm


# ------------------------------------------------------------------ label generation
def sample_configs(n: int, seed: int, two_sided: bool = True):
    """Seeded lattice descriptions spanning the workloads' range (mu = 0 only
    when two_sided is False: label runs at mu != 0 are switched off)."""
    rng = np.random.default_rng(seed)
    shapes = [(6, 6, 6, 6), (8, 8, 8, 8), (10, 10, 10, 10), (6, 6, 6, 12), (8, 8, 8, 12)]
    out = []
    for i in range(n):
        dims = shapes[int(rng.integers(len(shapes)))]
        mu = float(rng.choice([0.0, 0.0, 0.1, 0.2, 0.3]))
        if not two_sided:
            mu = 0.0
        out.append(dict(dims=dims, eps=float(rng.uniform(0.15, 0.45)), m0=float(rng.uniform(1.3, 1.8)), mu=mu,
                        seed=int(seed * 1000 + i), k=1200 if mu == 0.0 else 1000))
    return out


def label_configs(ctx, cfgs, sources_per_lattice: int = 4, log=None):
    """Label rows for every (config, source) pair; returns rows, k_refs, group ids."""
    import nks_inputs as I
    from . import Lattice, policy_label
    rows, krefs, groups = [], [], []
    batch = []

    def flush():
        if not batch:
            return
        t0 = time.time()
        lab = policy_label([dict(lat=lat, b=b, k=k, ell=256, tol=1e-8) for lat, b, k, _ in batch])
        for (lat, b, k, g), row in zip(batch, lab):
            rows.append(row)
            krefs.append(k)
            groups.append(g)
        if log:
            log(f"[policy] labelled {len(batch)} jobs in {time.time() - t0:.1f}s (total {len(rows)})")
        batch.clear()

    lats = []
    for gi, c in enumerate(cfgs):
        rng = np.random.default_rng(c["seed"] + 17)
        lat = Lattice(ctx, c["dims"], I.su3_links(c["dims"], c["eps"], c["seed"]), m0=c["m0"], mu=c["mu"])
        lats.append(lat)
        V = int(np.prod(c["dims"]))
        for s in range(sources_per_lattice):
            if s == sources_per_lattice - 1:
                b = I.gaussian_source(c["dims"], c["seed"] + 99)
            else:
                b = I.point_source(c["dims"], int(rng.integers(4)), int(rng.integers(3)), int(rng.integers(V)))
            batch.append((lat, b, c["k"], gi))
        if len(batch) >= 48 or sum(12 * lat_.V * k_ * 16 for lat_, _, k_, _ in batch) > 48e9:
            flush()
            lats.clear()
    flush()
    return np.asarray(rows), np.asarray(krefs), np.asarray(groups)


def compare(ctx, cfgs, tols=(1e-8, 1e-10), sources: int = 2, log=None):
    """Run the plain (DOUBLING) and the learned policies on the same jobs,
    one job per call; returns records with k_used, ell_used, status and the
    device time of each call (outer loop with checkpoints, nested step, lift)."""
    import nks_inputs as I
    from . import POLICY_DOUBLING, POLICY_LEARNED, Lattice, sign_apply
    out = []
    for c in cfgs:
        lat = Lattice(ctx, c["dims"], I.su3_links(c["dims"], c["eps"], c["seed"]), m0=c["m0"], mu=c["mu"])
        rng = np.random.default_rng(c["seed"] + 5)
        V = int(np.prod(c["dims"]))
        bs = [I.point_source(c["dims"], int(rng.integers(4)), int(rng.integers(3)), int(rng.integers(V))).ravel()
              for _ in range(sources)]
        for tol in tols:
            for b in bs:
                rec = dict(cfg=c, tol=tol)
                xs = {}
                for name, pol in (("plain", POLICY_DOUBLING), ("learned", POLICY_LEARNED)):
                    sign_apply(lat, b, k=1400, ell=256, tol=tol, k_policy=pol, ell_policy=pol)    # warm-up
                    x, st = sign_apply(lat, b, k=1400, ell=256, tol=tol, k_policy=pol, ell_policy=pol)
                    rec[name] = dict(k=st["k_used"], ell=st["ell_used"], status=st["status"],
                                     ms=st["ms_outer"] + st["ms_nested"] + st["ms_lift"])
                    xs[name] = x.cpu().numpy()
                rec["rel_learned_vs_plain"] = float(np.linalg.norm(xs["learned"] - xs["plain"]) /
                                                    np.linalg.norm(xs["plain"]))
                out.append(rec)
                if log:
                    log(f"[policy] {c['dims']} eps {c['eps']:.2f} m0 {c['m0']:.2f} mu {c['mu']} tol {tol:g}: "
                        f"k {rec['plain']['k']} -> {rec['learned']['k']}, ell {rec['plain']['ell']} -> "
                        f"{rec['learned']['ell']}, ms {rec['plain']['ms']:.1f} -> {rec['learned']['ms']:.1f}, "
                        f"status {rec['plain']['status']}/{rec['learned']['status']}, "
                        f"rel diff {rec['rel_learned_vs_plain']:.1e}")
        lat.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--lattices", type=int, default=120)
    ap.add_argument("--seed", type=int, default=31)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--labels", default=None, help="save/load the label rows here (.npz)")
    ap.add_argument("--compare", type=int, default=0, help="held-out lattices for a plain-vs-learned comparison")
    args = ap.parse_args(argv)
    import paper_0912_4457_amd as nks

    def log(m):
        print(m, flush=True)

    ctx = nks.Context(0)
    cfgs = sample_configs(args.lattices, args.seed, two_sided=False)
    if args.labels and os.path.exists(args.labels):
        z = np.load(args.labels)
        rows, krefs, groups = z["rows"], z["krefs"], z["groups"]
    else:
        rows, krefs, groups = label_configs(ctx, cfgs, log=log)
        if args.labels:
            np.savez(args.labels, rows=rows, krefs=krefs, groups=groups)
    X, T, G = dataset(rows, krefs, groups)
    log(f"[policy] {len(rows)} label rows -> {len(X)} samples")
    held = G % 5 == 0                                   # every fifth lattice is held out
    fm, fs, tm, ts = normalisation(X[~held], T[~held])
    params, hist = train(ctx, (X[~held] - fm) / fs, (T[~held] - tm) / ts, steps=args.steps, seed=args.seed, log=log)
    pred = predict(ctx, params, fm, fs, tm, ts, X[held])
    res = T[held] - pred
    shift = float(np.quantile(res[:, 0], 0.85)) if len(res) else 0.0
    shift_ell = float(np.quantile(res[:, 1], 0.10)) if len(res) else 0.0
    tm_shift = tm.copy()
    tm_shift[0] += max(shift, 0.0)
    tm_shift[1] += min(shift_ell, 0.0)
    rms = np.sqrt(np.mean(res ** 2, axis=0)) if len(res) else np.zeros(2)
    meta = dict(samples_train=int((~held).sum()), samples_held=int(held.sum()), label_rows=int(len(rows)),
                lattices=args.lattices, seed=args.seed, steps=args.steps, loss=hist,
                held_rms_log10_k=float(rms[0]), held_rms_log10_ell=float(rms[1]), k_shift_log10=max(shift, 0.0),
                ell_shift_log10=min(shift_ell, 0.0),
                tols=list(TOLS))
    log(f"[policy] held-out rms log10 k {rms[0]:.4f}, log10 ell {rms[1]:.4f}, k shift {shift:.4f}")
    blob = pack(params, fm, fs, tm_shift, ts)
    if args.compare:
        from . import policy_load
        policy_load(ctx, blob)
        recs = compare(ctx, sample_configs(args.compare, args.seed + 1), log=log)
        kp = sum(r["plain"]["k"] for r in recs)
        kl = sum(r["learned"]["k"] for r in recs)
        mp = sum(r["plain"]["ms"] for r in recs)
        ml = sum(r["learned"]["ms"] for r in recs)
        meta["compare"] = dict(lattices=args.compare, k_plain=kp, k_learned=kl, ms_plain=mp, ms_learned=ml,
                               max_rel_learned_vs_plain=max(r["rel_learned_vs_plain"] for r in recs))
        log(f"[policy] held-out comparison: sum k {kp} -> {kl} ({kl / kp:.3f}), device ms {mp:.1f} -> {ml:.1f}")
    save(args.out, blob, meta)
    log(f"[policy] wrote {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
