"""Error measures of the parity tests (FP64).  Element-wise relative to |A||x| for products,
normwise plus residual for solves.  The oracle supplies the absolute-value products."""
import numpy as np

import oracle as O

TOL = 1e-12
RES_TOL = 1e-14


def _abs(A):
    from types import SimpleNamespace
    return SimpleNamespace(n_rows=A.n_rows, n_cols=A.n_cols, row_ptr=A.row_ptr, col_idx=A.col_idx,
                           values=np.abs(A.values))


def check_product(A, X, got, ref):
    """max_i |got_i - ref_i| / (|A||X|)_i <= TOL; rows with (|A||X|)_i = 0 must be exactly 0."""
    scale = O.spmv(_abs(A), np.abs(X))
    err = np.abs(got - ref)
    zero = scale == 0
    assert np.all(got[zero] == 0), "nonzero output where |A||x| = 0"
    rel = np.max(err[~zero] / scale[~zero]) if np.any(~zero) else 0.0
    assert rel <= TOL, f"elementwise relative error {rel:.3e}"
    return rel


def check_gv(A, X, G, got, ref, sign=1.0):
    """GV[e] against sum_r |g_i x_j|."""
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    scale = np.sum(np.abs(G[rows]) * np.abs(X[A.col_idx]), axis=1)
    err = np.abs(got - ref)
    zero = scale == 0
    assert np.all(got[zero] == 0)
    rel = np.max(err[~zero] / scale[~zero]) if np.any(~zero) else 0.0
    assert rel <= TOL, f"gv elementwise relative error {rel:.3e}"
    return rel


def check_solve(L, B, got, ref, transposed=False):
    """||got - ref||_inf / ||ref||_inf <= TOL and residual <= RES_TOL."""
    nrm = np.max(np.abs(ref)) if ref.size else 0.0
    err = np.max(np.abs(got - ref)) if ref.size else 0.0
    assert err <= TOL * max(nrm, np.finfo(float).tiny), f"normwise error {err / max(nrm, 1e-300):.3e}"
    if transposed:
        LT, _ = O.transpose(L)
        Lmat = LT
    else:
        Lmat = L
    r = B - O.spmv(Lmat, got)
    scale = np.max(O.spmv(_abs(Lmat), np.abs(got))) + np.max(np.abs(B)) if B.size else 1.0
    res = np.max(np.abs(r)) / scale if B.size else 0.0
    assert res <= RES_TOL, f"residual {res:.3e}"
    return err / max(nrm, 1e-300), res


def check_gv_solve(L, X, lam_dev, lam_ref, got, ref):
    """GV of the solve adjoint, GV[e] = -sum_r lam[i,r] X[j,r].  (1) The GV pass itself,
    against the device's own lambda, elementwise within 1e-14 of sum_r |lam_i x_j|; (2) the
    propagated error of lambda: |got - ref| <= TOL * ||lam||_inf * sum_r |X[j, r]|."""
    rows = np.repeat(np.arange(L.n_rows), np.diff(L.row_ptr))
    cols = L.col_idx
    own = -np.sum(lam_dev[rows] * X[cols], axis=1)
    scale = np.sum(np.abs(lam_dev[rows]) * np.abs(X[cols]), axis=1)
    err = np.abs(got - own)
    assert np.all(err <= 1e-14 * scale + 0.0), f"GV pass error {np.max(err / np.maximum(scale, 1e-300)):.3e}"
    bound = TOL * np.max(np.abs(lam_ref)) * np.sum(np.abs(X[cols]), axis=1)
    assert np.all(np.abs(got - ref) <= bound), "GV propagated error above bound"
