"""Writes sdp_optima.json: the optimum of min <c, x> over each spectrahedron of
the annealing workload (S-n-n of the paper's generator, n = 30, 40, 50, 60,
ten each, seeded objectives), computed by the oracle's log-barrier method to a
duality gap of 1e-10 relative.  Run from the repository root:
    python tests/golden/make_sdp_optima.py"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.sdp_barrier import sdp_min  # noqa: E402
from paper_2010_03817_amd import instances as I  # noqa: E402


def main():
    out = []
    for n, iseed, cseed in I.sdp_family():
        inst = I.paper_random(n, n, seed=iseed)
        c = I.objective(n, cseed)
        _, f, t = sdp_min(inst, c, gap=1e-10)
        out.append({"n": n, "m": n, "instance_seed": iseed, "objective_seed": cseed, "f_star": f,
                    "barrier_t": t})
        print(n, iseed, f, flush=True)
    doc = {"citation": "the optimisation section of the paper (eq. (sdp)); instances of its random generator "
                       "(Section 4) as in its annealing table, objectives seeded unit vectors",
           "method": "oracle/sdp_barrier.py: primal log-barrier path following, gap M/t <= 1e-10 max(1, |f|)",
           "optima": out}
    with open(os.path.join(HERE, "sdp_optima.json"), "w") as fh:
        json.dump(doc, fh, indent=1)


if __name__ == "__main__":
    main()
