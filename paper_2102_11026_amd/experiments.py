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


def fd_vs_csfd(nmr, ctx, steps: int = 15, iters: int = 6, hs=(1e-3, 1e-5, 1e-7, 1e-9),
               precs=("fp32", "fp64")) -> dict:
    """The comparison of complex steps with recursive central differences
    (Sec. 6) on the fast-motion problem of synth.lsd_problem: for each
    precision and step h, the error of J and dJ against the complex-step
    values at the initial state, then `steps` implicit-Euler steps with the
    central-difference derivatives in the Newton iteration.  Reported per run:
    its status, the steps it completed, the largest relative deviation of r
    from the complex-step run, and the largest ratio of the last to the first
    Newton residual of a step (complex steps reach about 1e-12)."""
    p = synth.lsd_problem()
    rng = np.random.default_rng(21)
    q = p.r0[p.n_p:] + rng.normal(size=p.n_q) * 0.05
    dq, qd = rng.normal(size=p.n_q) * 0.02, rng.normal(size=p.n_q) * 0.5
    rel = lambda a, b: float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))
    out = dict(problem=p.name, steps=steps, newton_iters=iters, runs=[])
    for prec in precs:
        ref = nmr.Instance(ctx, p, prec)
        try:
            d_ref = ref.decoder_jacobian_hessian(q, dq, qd)
            J_ref, dJ_ref = d_ref["J"].cpu().numpy(), d_ref["dJ"].cpu().numpy()
            traj = []
            for _ in range(steps):
                ref.step(iters, resid=False)
                traj.append(ref.get_state()[0])
        finally:
            ref.close()
        for h in hs:
            x = nmr.Instance(ctx, p.replace(fd_h=h), prec)
            row = dict(precision=prec, h=h)
            try:
                d = x.decoder_jacobian_hessian(q, dq, qd)
                row["J_rel_err"] = rel(d["J"].cpu().numpy(), J_ref)
                row["dJ_rel_err"] = rel(d["dJ"].cpu().numpy(), dJ_ref)
                dev, done, ratio, status = 0.0, 0, None, "ok"
                for k in range(steps):
                    try:
                        norms = x.step(iters)
                    except nmr.NmrError as e:
                        status = nmr.STATUS.get(e.code, str(e.code))
                        break
                    r = x.get_state()[0]
                    if not np.all(np.isfinite(r)):
                        status = "nonfinite"
                        break
                    done = k + 1
                    dev = max(dev, rel(r, traj[k]))
                    ratio = max(ratio or 0.0, float(norms[-1] / max(norms[0], 1e-300)))
                row.update(status=status, steps_completed=done, max_r_rel_dev=dev, worst_newton_ratio=ratio)
            finally:
                x.close()
            out["runs"].append(row)
    return out
