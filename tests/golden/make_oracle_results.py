"""Writes the oracle's end points for the seeded parity workloads.

    python tests/golden/make_oracle_results.py            # small cases
    python tests/golden/make_oracle_results.py --large    # full-size cases

Calls only oracle/ (and the seeded input generators).  Output:
tests/golden/oracle_results.json (small cases) or
tests/golden/oracle_results_large.json (the n=100 system, held-out members of
the n=32 warm-start family and the largest members of the mixed batch, each
solved in the oracle's expanded Schur mode), with, per case, the verdict,
objectives, duality gap, the certificate margins and the phase-I optimum,
which the GPU parity tests compare against.  The large file is rewritten
after every case, so an interrupted run keeps what it finished.
"""
import json
import os
import sys
import time
from math import comb

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ipm, sdp as S  # noqa: E402
from paper_1411_3769_amd import workloads as W  # noqa: E402


MIXED_MAX_K = 300


def mixed_K(sy):
    return comb(sy.l + sy.dp - 1, sy.dp) * sy.n * (sy.n + 1) // 2


def run(sy):
    sdp = S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d)
    t = time.time()
    r = ipm.ipm_solve(sdp)
    return dict(tag=sy.tag, seed=sy.seed, n=sy.n, l=sy.l, dp=sy.dp, d=sy.d,
                verdict=ipm.VERDICT_NAMES[r.verdict], reason=ipm.REASON_NAMES[r.reason],
                iterations=r.iterations, phi=r.phi, psi=r.psi, gap_rel=r.gap_rel, pinf=r.pinf,
                dinf=r.dinf, margin=r.margin, margin_P=r.margin_P, margin_D=r.margin_D,
                phase1_used=r.phase1_used, phase1_iterations=r.phase1_iterations,
                t_star=r.t_star, seconds=time.time() - t)


LARGE_MIXED = (200, 36)   # K = 17640 (the batch's largest) and K = 2583


def main_large():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_results_large.json")
    out = []
    if os.path.exists(path):
        with open(path) as fh:
            out = json.load(fh)
    have = {(r["tag"], r["seed"]) for r in out}
    mixed = W.mixed_systems(512)
    cases = [W.c2_system(0)] + [W.warm_system(10**6 + s) for s in range(8)]
    cases += [mixed[i] for i in LARGE_MIXED]
    for sy in cases:
        if (sy.tag, sy.seed) in have:
            continue
        rec = run(sy)
        if rec["tag"].startswith("mixed"):
            rec["index"] = int(rec["tag"][5:])
        out.append(rec)
        print(rec["tag"], rec["seed"], rec["verdict"], rec["iterations"], f"{rec['seconds']:.2f}s",
              flush=True)
        with open(path + ".tmp", "w") as fh:
            json.dump(out, fh, indent=1)
        os.replace(path + ".tmp", path)


def main():
    if "--large" in sys.argv[1:]:
        return main_large()
    cases = []
    for s in range(16):
        cases.append(W.plain_system(s))
        cases.append(W.plain_system(s, twin=True))
    for s in range(64):
        cases.append(W.c1_system(s))
    for (n, l) in [(4, 5), (5, 6), (7, 8), (16, 3), (24, 2)]:
        cases.append(W.paper_shape_system(n, l, 0))
    # the members of the 512-system mixed batch small enough for the oracle
    for i, sy in enumerate(W.mixed_systems(512)):
        if mixed_K(sy) <= MIXED_MAX_K:
            cases.append(sy)
    out = []
    for sy in cases:
        rec = run(sy)
        if rec["tag"].startswith("mixed"):
            rec["index"] = int(rec["tag"][5:])
        out.append(rec)
        print(rec["tag"], rec["seed"], rec["verdict"], rec["iterations"], f"{rec['seconds']:.2f}s",
              flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_results.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
