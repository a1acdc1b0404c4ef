"""Experiments on the finished Newton path (run through the C ABI on the GPU).

consistency_in_dt: the paper's formulation keeps the fictitious force
f_fict = M H(dq, dq) (eq. fict) and its derivative in the Newton matrix; the
trimmed formulation drops it, as latent space dynamics does (Sec. 3.3, and
the comparison with it in Sec. 6).  With f_fict the scheme is implicit Euler
on J q'' + H(q', q') = M^-1 (f_ext - f_int) projected on the tangent space, so
its trajectory converges to the fine-step reference as dt -> 0; without it
the discrete equations approximate a different ODE (the H(q', q') term does
not vanish with dt), so the error stops decreasing under fast motion.  The
experiment integrates the fast-motion problem of synth.lsd_problem to a fixed
time at dt = 1/60, 1/120, ... with enough Newton iterations to converge, and
reports the relative error of u(T) against the paper's formulation at a much
smaller step.
"""
from __future__ import annotations

import numpy as np

from . import synth


def _integrate(nmr, ctx, p, prec, dt, T, iters):
    steps = int(round(T / dt))
    inst = nmr.Instance(ctx, p.replace(dt=dt), prec)
    try:
        st, _ = nmr.step_many(ctx, [inst], steps, iters)
        r, _, u = inst.get_state(with_u=True)
    finally:
        inst.close()
    return st[0], np.asarray(u, np.float64), steps


def consistency_in_dt(nmr, ctx, prec: str = "fp64", T: float = 0.25, levels: int = 5, ref_level: int = 7,
                      iters: int = 6) -> dict:
    """Relative error of u(T) for both formulations at dt = 1/(60 2^k),
    k < levels, against the paper's formulation at k = ref_level."""
    p = synth.lsd_problem()
    st, u_ref, n_ref = _integrate(nmr, ctx, p, prec, 1.0 / (60 * 2 ** ref_level), T, iters)
    assert st == 0, st
    out = dict(problem=p.name, precision=prec, T=T, newton_iters=iters, reference_dt=f"1/{60 * 2 ** ref_level}",
               reference_steps=n_ref, levels=[])
    for k in range(levels):
        dt = 1.0 / (60 * 2 ** k)
        row = dict(dt=f"1/{60 * 2 ** k}")
        for form in ("full", "trimmed"):
            st, u, _ = _integrate(nmr, ctx, p.replace(formulation=form), prec, dt, T, iters)
            row[form] = float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)) if st == 0 else None
            row[form + "_status"] = st
        out["levels"].append(row)
    return out
