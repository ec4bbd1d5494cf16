"""The shifted solve (Q - tau I) x = b in its Gamma5-preconditioned form.

eq. (3.6) <=> eq. (3.7): (Q - tau I) x = b  <=>  (D - tau Gamma5) x = Gamma5 b,
solved with FGMRES (Sec. 2, multigrid as a preconditioner of a flexible Krylov
method) preconditioned by the two-level V-cycle, or by SAP alone when no
coarse level is given (the coarse-correction-off variant of Sec. 4).
Because Gamma5 is a sign flip, ||b - (Q - tau) x|| = ||Gamma5 b - A_tau x||.
"""
from .dirac import gamma5
from .krylov import fgmres
from .sap import sap


def solve_shifted(op, b, tau, block, mg=None, tol=1e-10, restart=8, maxiter=500,
                  nu=3, n_mr=3, coarse_iters=50, coarse_tol=0.5, qform=False, smoother="sap"):
    """qform: solve (Q - tau) x = b directly, every level built on Q - tau (the
    comparison of Sec. 3.3) instead of the Gamma5-preconditioned form."""
    f = b.copy() if qform else gamma5(b)

    def A(v):
        av = op.A(v, tau)
        return gamma5(av) if qform else av

    if mg is not None:
        def M(v):
            return mg.vcycle(v, tau, nu, n_mr, coarse_iters, coarse_tol, qform, smoother)
    else:
        def M(v):
            return sap(op, v, 0.0 * v, tau, block, nu, n_mr, qform)

    return fgmres(A, M, f, tol, restart, maxiter)
