"""How far the workloads' stop tolerances leave a step from its exact root (test
infrastructure: a report, run by hand; nothing in the library imports it).

For each named workload, Algorithm 1 of the oracle is run from the workload's initial
state to the workload's tolerance, and its result is compared, point by point, with a
reference root: the damped Newton root with a direct solve (newton.py) where the
system is small enough, else the oracle's own Algorithm 1 run to a tolerance near the
FP64 round-off floor of the plain norm (Sec. 2.1 stopping criterion; the step's root
is unique for these parameters, so both references are the same point up to that
floor).

    python tests/root_distance.py ac64 ch512 schnak1024:1e-7 ac2048:1e-8

Each argument is a workload name, optionally followed by ":tol" to use the tight
Algorithm-1 reference at that tolerance instead of Newton.  Prints one JSON line per
workload.
"""
import json
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import numpy as np

from oracle import equations as oeq, newton, pdhg
from paper_2305_03945_amd import workloads as wl


def problem_of(cfg):
    return oeq.Problem(kind=cfg["kind"], N=cfg["N"], L=cfg.get("L", 1.0), bc=cfg["bc"], diff=tuple(cfg["diff"]),
                       b=cfg.get("b", 1.0), a=cfg.get("a", 0.0), sb=cfg.get("sb", 0.0),
                       kappa=cfg.get("kappa", 1.0), dim=cfg.get("dim", 2))


def options_of(cfg, tol=None, max_iter=10000):
    tau = cfg.get("tau", 0.9)
    return pdhg.Options(tol=cfg["tol"] if tol is None else tol, max_iter=max_iter, tau_u=tau, tau_p=tau,
                        omega=cfg.get("omega", 1.0))


def report(name, ref_tol=None):
    cfg = wl.CONFIGS[name]
    prob = problem_of(cfg)
    U0 = wl.initial_field(cfg)
    t0 = time.time()
    r = pdhg.step(prob, U0, cfg["ht"], options_of(cfg))
    if ref_tol is None:
        root = newton.root(prob, U0, cfg["ht"]).U
        how = "newton"
    else:
        root = pdhg.step(prob, U0, cfg["ht"], options_of(cfg, tol=ref_tol, max_iter=100000)).U
        how = "algorithm 1 to %g" % ref_tol
    return dict(workload=name, tol=cfg["tol"], iters=r.iters, reference=how,
                maxabs_to_root=float(np.max(np.abs(r.U - root))), seconds=round(time.time() - t0, 1))


def main(argv):
    for a in argv:
        name, _, tol = a.partition(":")
        print(json.dumps(report(name, float(tol) if tol else None)), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
