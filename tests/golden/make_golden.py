"""Write the stored expected values of the parity tests.

Every number written here comes from the CPU oracle (``oracle/``) run on the
seeded synthetic workloads of ``synth``; nothing comes from the GPU library.
The solve is run to the rounding floor (the oracle's stall rule) in chunks of
warm-started iterations so a long run can resume from its last state.

    python tests/golden/make_golden.py chain40
    python tests/golden/make_golden.py chain2k --state-dir /tmp/golden_state

Output: tests/golden/<workload>.json with the converged objective f*, the
iteration count, the nonzero counts, and the supports {|x| > 1e-6} of Lambda*
and Theta* as zlib-compressed bitmasks (numpy.packbits, row-major).

A run too long to reach the floor can be summarised from its saved state:

    python tests/golden/make_golden.py chain2k --state-dir /tmp/golden_state \
        --tail-estimate --note "how the state was produced"

writes tests/golden/<workload>_tail.json: the oracle's objective at the saved
iterate (an upper bound on f*, recomputed here by the oracle), the per-
iteration decreases of f over the last iterations, and f* extrapolated from
them as a geometric tail (the decrease shrinks by a fitted factor r per
iteration, so the remaining gap is d_last * r / (1 - r)), fitted over the
last 10, 20, 40 and 80 decreases; the spread of those four extrapolations is
the estimate's stated uncertainty.  This is an extrapolation, not the
optimum: it pins a solve's limit only as closely as the tail is geometric.
"""
import argparse
import base64
import json
import os
import sys
import time
import zlib

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

SUPPORT_EPS = 1e-6


def pack_mask(mask: np.ndarray) -> str:
    return base64.b64encode(zlib.compress(np.packbits(mask.reshape(-1)).tobytes(), 9)).decode()


def unpack_mask(s: str, shape) -> np.ndarray:
    bits = np.frombuffer(zlib.decompress(base64.b64decode(s)), np.uint8)
    return np.unpackbits(bits)[: int(np.prod(shape))].reshape(shape).astype(bool)


def load(name: str) -> dict:
    with open(os.path.join(HERE, f"{name}.json")) as fh:
        g = json.load(fh)
    q, p = g["q"], g["p"]
    g["support_Lambda"] = unpack_mask(g["support_Lambda"], (q, q))
    g["support_Theta"] = unpack_mask(g["support_Theta"], (p, q))
    g["borderline_Lambda"] = unpack_mask(g["borderline_Lambda"], (q, q))
    g["borderline_Theta"] = unpack_mask(g["borderline_Theta"], (p, q))
    return g


TAIL_WINDOWS = (10, 20, 40, 80)


def fit_tail(f):
    """Geometric-tail extrapolations of the limit of a decreasing sequence f:
    for each window w, the factor r by which the last w decreases shrink
    (least squares on their logarithms) and f[-1] - d_last r / (1 - r)."""
    f = np.asarray(f, dtype=np.float64)
    d = -np.diff(f)
    assert d.size >= max(TAIL_WINDOWS), "too short a sequence"
    assert (d[-max(TAIL_WINDOWS):] > 0).all(), "the tail is not strictly decreasing"
    fits = []
    for w in TAIL_WINDOWS:
        rate = float(np.exp(np.polyfit(np.arange(w), np.log(d[-w:]), 1)[0]))
        assert rate < 1.0
        gap = float(d[-1] * rate / (1.0 - rate))
        fits.append({"window": w, "rate": rate, "gap": gap, "f_star": float(f[-1]) - gap})
    return fits


def tail_estimate(args, pr):
    """Summarise a saved oracle run (see the module docstring)."""
    state = args.state_dir
    Lam = np.load(os.path.join(state, "Lambda.npy"))
    Th = np.load(os.path.join(state, "Theta.npy"))
    meta = json.load(open(os.path.join(state, "meta.json")))
    done, fs = meta["done"], meta["f"]
    assert len(fs) == done, "state trace and iteration count disagree"
    f_K = oracle.objective(oracle.stats(pr.X, pr.Y), Lam, Th, pr.lam_Lambda, pr.lam_Theta)
    assert f_K is not None, "saved Lambda is not positive definite"
    f = np.array(fs + [f_K])          # f at the top of iterations 0 .. done
    d = -np.diff(f)
    fits = fit_tail(f)
    est = [x["f_star"] for x in fits]
    out = {
        "workload": args.workload, "seed": args.seed, "n": pr.n, "p": pr.p, "q": pr.q,
        "name": pr.name, "lam_Lambda": pr.lam_Lambda, "lam_Theta": pr.lam_Theta,
        "iterations": done, "f_K": f_K,
        "decreases_tail": [float(x) for x in d[-max(TAIL_WINDOWS):]],
        "fits": fits,
        "f_star_estimate": fits[0]["f_star"],
        "f_star_spread": float(max(est) - min(est)),
        "nnz_Lambda": int(np.count_nonzero(np.abs(Lam) > SUPPORT_EPS)),
        "nnz_Theta": int(np.count_nonzero(np.abs(Th) > SUPPORT_EPS)),
        "f_trace_head": fs[:50],
        "generator": "synth.workload(%r, seed=%r) -> oracle.solve(tol=%g, stall_iters=3), "
                     "warm-started chunks; %s" % (args.workload, args.seed, args.tol, args.note),
    }
    with open(os.path.join(HERE, f"{args.workload}_tail.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {args.workload}_tail: K={done} f_K={f_K!r} f* ~ {out['f_star_estimate']!r} "
          f"spread {out['f_star_spread']:.3e}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(synth.WORKLOADS))
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--chunk", type=int, default=25)
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--state-dir", default=None)
    ap.add_argument("--lambda-passes", type=int, default=1)
    ap.add_argument("--tol", type=float, default=0.0,
                    help="stop also when the subgradient is below tol (||Lambda||_1 + "
                         "||Theta||_1) (0: only at the rounding floor of f)")
    ap.add_argument("--tail-estimate", action="store_true",
                    help="summarise the saved state of --state-dir instead of iterating")
    ap.add_argument("--note", default="",
                    help="with --tail-estimate: how the saved state was produced")
    args = ap.parse_args()
    pr = synth.workload(args.workload, seed=args.seed)
    if args.tail_estimate:
        tail_estimate(args, pr)
        return
    state = args.state_dir
    Lam = Th = None
    done = 0
    fs = []
    if state and os.path.exists(os.path.join(state, "Lambda.npy")):
        Lam = np.load(os.path.join(state, "Lambda.npy"))
        Th = np.load(os.path.join(state, "Theta.npy"))
        meta = json.load(open(os.path.join(state, "meta.json")))
        done, fs = meta["done"], meta["f"]
    t0 = time.time()
    while True:
        r = oracle.solve(pr.X, pr.Y, pr.lam_Lambda, pr.lam_Theta, tol=args.tol,
                         max_iter=args.chunk, stall_iters=3, Lambda0=Lam, Theta0=Th,
                         lambda_passes=args.lambda_passes)
        Lam, Th = r.Lambda, r.Theta
        done += r.iters
        fs.extend(float(v) for v in r.trace["f"][: r.iters])
        print(f"[{time.time() - t0:9.1f}s] iters={done} f={r.f!r} "
              f"subgrad/l1={r.trace['subgrad'][-1] / r.trace['l1'][-1]:.3e} status={r.status}",
              flush=True)
        if state:
            os.makedirs(state, exist_ok=True)
            np.save(os.path.join(state, "Lambda.npy"), Lam)
            np.save(os.path.join(state, "Theta.npy"), Th)
            json.dump({"done": done, "f": fs}, open(os.path.join(state, "meta.json"), "w"))
        if r.status in (oracle.ORC_STALLED, oracle.ORC_OK) or done >= args.max_iter:
            break
    out = {
        "workload": args.workload, "seed": args.seed, "n": pr.n, "p": pr.p, "q": pr.q,
        "name": pr.name,
        "lam_Lambda": pr.lam_Lambda, "lam_Theta": pr.lam_Theta,
        "f_star": r.f, "iterations": done, "status": int(r.status),
        "subgrad_l1": float(r.trace["subgrad"][-1]), "l1": float(r.trace["l1"][-1]),
        "nnz_Lambda": int(np.count_nonzero(np.abs(Lam) > SUPPORT_EPS)),
        "nnz_Theta": int(np.count_nonzero(np.abs(Th) > SUPPORT_EPS)),
        "support_eps": SUPPORT_EPS,
        "support_Lambda": pack_mask(np.abs(Lam) > SUPPORT_EPS),
        "support_Theta": pack_mask(np.abs(Th) > SUPPORT_EPS),
        # entries whose magnitude lies in [1e-7, 1e-5]: support comparisons skip them
        "borderline_Lambda": pack_mask((np.abs(Lam) >= 1e-7) & (np.abs(Lam) <= 1e-5)),
        "borderline_Theta": pack_mask((np.abs(Th) >= 1e-7) & (np.abs(Th) <= 1e-5)),
        "f_trace_head": fs[:50],
        "generator": "synth.workload(%r, seed=%r) -> oracle.solve(tol=%g, stall_iters=3, "
                     "lambda_passes=%d)" % (args.workload, args.seed, args.tol,
                                            args.lambda_passes),
    }
    with open(os.path.join(HERE, f"{args.workload}.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", args.workload, "f*", r.f)


if __name__ == "__main__":
    main()
