"""Shared helpers of the GPU tests: build matching oracle and ABI problems from a
workload description.  (Test infrastructure; imports the oracle.)"""
import numpy as np

from oracle import equations as oeq, pdhg as opdhg
from paper_2305_03945_amd import workloads as wl


def oracle_problem(cfg, N=None, bc=None):
    return oeq.Problem(kind=cfg["kind"], N=N or cfg["N"], L=cfg.get("L", 1.0), bc=bc or cfg["bc"],
                       diff=tuple(cfg["diff"]), b=cfg.get("b", 1.0), a=cfg.get("a", 0.0), sb=cfg.get("sb", 0.0),
                       kappa=cfg.get("kappa", 1.0), dim=cfg.get("dim", 2))


def oracle_opts(cfg, tol=None, max_iter=10000, init="prev"):
    tau = cfg.get("tau", 0.9)
    return opdhg.Options(tol=cfg["tol"] if tol is None else tol, max_iter=max_iter, tau_u=tau, tau_p=tau,
                         omega=cfg.get("omega", 1.0), init=init)


def small_cfg(kind, N, bc):
    """Parameters of the named configuration of this equation, on an N x N grid."""
    name = {"allen_cahn": "ac2048", "cahn_hilliard": "ch512", "schnakenberg": "schnak1024"}[kind]
    cfg = dict(wl.CONFIGS[name])
    cfg.update(N=N, bc=bc)
    return cfg


def max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))
