"""Adaptive time step size around the implicit step (FP64, test only).

Sec. 2.2 ("Adaptive time stepsize"): the PDHG solve of a step converges only
below a threshold step size that changes during the run, so the step size is
adapted from the PDHG iteration count M of each step.  With an upper bound
h_t^0 (also the first step size), thresholds N^* > N_* > 0 and a factor
eta in (0, 1), the step size for the next step is

    M > N^*          ->  eta h_t                         (shrink)
    N_* <= M <= N^*  ->  h_t                             (keep)
    M < N_*          ->  h_t / eta if that is <= h_t^0,  (enlarge)
                         else h_t

Readings taken here (the paper is silent on them):

* A step whose solve did not converge (iteration limit reached, or the residual
  non-finite / diverging) is rejected: the state is kept and the step is
  retried with eta h_t.  An accepted step always advances the state, also when
  its M exceeds N^* (the paper resets h_t "for the next time step").
* The last step is shortened to land on t_end: h = min(h_t, t_end - t), and the
  rule acts on the step size actually used.  The run ends when
  t_end - t <= 1e-14 max(1, |t_end|).
* A retry below h_min, or more than max_rejects consecutive rejections, ends the
  run with status "noconv".

The oracle's state updates use only FP64 additions and multiplications in the
order written, so an implementation that makes the same decisions from the same
iteration counts reproduces the step-size sequence bit for bit.
"""
from dataclasses import dataclass, field

from . import pdhg


@dataclass
class Adapt:
    ht0: float
    eta: float = 0.75
    n_hi: int = 100          # N^*
    n_lo: int = 20           # N_*
    ht_min: float = 1e-12
    max_rejects: int = 30


def next_step(a, ht, iters, status):
    """(h_t for the next attempt, whether this step is accepted)."""
    if status != pdhg.OK:
        return a.eta * ht, False
    if iters > a.n_hi:
        return a.eta * ht, True
    if iters < a.n_lo:
        up = ht / a.eta
        return (up if up <= a.ht0 else ht), True
    return ht, True


@dataclass
class AdvanceResult:
    U: object
    t: float
    ht: float
    status: str
    accepted: int = 0
    rejected: int = 0
    shrinks: int = 0
    enlarges: int = 0
    pdhg_iters: int = 0
    trace: list = field(default_factory=list)   # (h used, iterations, accepted)


def done_time(t, t_end):
    return t_end - t <= 1e-14 * max(1.0, abs(t_end))


def advance(prob, U, t_end, opts, a, t0=0.0):
    """Integrate from t0 to t_end with the adaptive rule, every step by Algorithm 1."""
    t, ht = t0, a.ht0
    res = AdvanceResult(U=U, t=t, ht=ht, status=pdhg.OK)
    rejects = 0
    while not done_time(t, t_end):
        h = min(ht, t_end - t)
        r = pdhg.step(prob, U, h, opts)
        res.pdhg_iters += r.iters
        nxt, ok = next_step(a, h, r.iters, r.status)
        res.trace.append((h, r.iters, ok))
        if ok:
            U = r.U
            t = t + h
            res.accepted += 1
            rejects = 0
        else:
            res.rejected += 1
            rejects += 1
        if nxt < h:
            res.shrinks += 1
        elif nxt > h:
            res.enlarges += 1
        ht = nxt
        if not ok and (ht < a.ht_min or rejects > a.max_rejects):
            res.status = pdhg.NOCONV
            break
    res.U, res.t, res.ht = U, t, ht
    return res
