"""CPU pin of the lagged CGS2 reading (DCGS2 of Swirydowicz, Langou,
Ananthan, Yang and Thomas, 2020, in GMRES(m) with a fixed preconditioner):
a numpy model of its recurrences (the once-projected vector u with norm eta,
the previous Hessenberg column made final from the next step's dot products,
the coefficients of the new column taken from those dot products and H
without another pass, the provisional column rotated for the estimate, the
cycle's last column used in its provisional form) against what GMRES must
produce by definition: the minimum residual over the Krylov space, formed
here by an explicit least-squares solve, plus the lucky breakdowns of
Algorithm 1 on eigenvectors and on identity plus rank 3, and the Arnoldi
relation with an orthonormal basis where one projection leaves visible
components along V.  The second-order parts of the lagged correction (|s|^2
in alpha^2, eta s in the previous column) are of rounding size whenever the
breakdown floor holds (s ~ eps |w| / eta), so no rounding-tolerant check
sees them; a wrong sign in d, a missing H s term or a missing second
projection of v_j each fail a test here.  The model is test code only; the
GPU kernels are checked against the oracle elsewhere."""
import numpy as np
import pytest

EPS = np.finfo(float).eps


def _rotate(col, cs, sn, upto):
    for k in range(upto):
        t = cs[k] * col[k] + sn[k] * col[k + 1]
        col[k + 1] = -sn[k] * col[k] + cs[k] * col[k + 1]
        col[k] = t


def lagged_gmres(A, Minv, b, m, maxit, rtol, keep=None):
    n = len(b)
    x = np.zeros(n)
    bn = np.linalg.norm(b)
    hist, its = [], 0
    while True:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if its == 0:
            hist.append(beta)
        if beta <= rtol * bn or its >= maxit:
            return x, hist, its
        V = np.zeros((n, m + 2))
        V[:, 0] = r / beta
        R = np.zeros((m + 1, m + 1))
        Hu = np.zeros((m + 1, m + 1))
        g = np.zeros(m + 2)
        g[0] = beta
        cs, sn = np.zeros(m + 1), np.zeros(m + 1)
        st = dict(eta=1.0, hp=np.zeros(m + 2), gsave=0.0)

        def column(jj, col, hn):   # rotations 0..jj-1, rotation jj, g
            col[jj + 1] = hn
            _rotate(col, cs, sn, jj)
            rr = np.hypot(col[jj], col[jj + 1])
            c, s = (col[jj] / rr, col[jj + 1] / rr) if rr else (1.0, 0.0)
            cs[jj], sn[jj] = c, s
            col[jj], col[jj + 1] = rr, 0.0
            R[:jj + 2, jj] = col[:jj + 2]
            g[jj + 1] = -s * g[jj]
            g[jj] = c * g[jj]

        def step(j):
            eta, hp = st["eta"], st["hp"]
            u, w = V[:, j].copy(), V[:, j + 1].copy()
            a, bb = V[:, :j + 1].T @ u, V[:, :j + 1].T @ w           # pass A
            ok = eta > 0
            s = a[:j] / eta if ok else np.zeros(j)
            sig = a[j] / eta ** 2 if ok else 0.0
            al2 = sig - s @ s
            ok = ok and al2 > 0.5 * sig
            al = np.sqrt(al2) if ok else 0.0
            if not ok:
                s = np.zeros(j)
            st["smax"] = max(st.get("smax", 0.0), float(np.abs(s).max()) if j else 0.0)
            if j >= 1:                                                 # column j-1 final
                col = np.zeros(j + 2)
                col[:j] = hp[:j] + (eta * s if ok else 0.0)
                col[j] = eta * al if ok else 0.0
                Hu[:j + 1, j - 1] = col[:j + 1]
                g[j - 1] = st["gsave"]
                column(j - 1, col, col[j])
            if ok:
                hs = Hu[:j + 1, :j] @ s
                bwj = (bb[j] / eta - s @ bb[:j]) / al
                h = (np.append(bb[:j], bwj) / eta - hs) / al
                d = hs / al + h
                cu = 1.0 / (eta * al)
                vj = cu * u - V[:, :j] @ (s / al)                      # pass B
                un = cu * w - V[:, :j] @ d[:j] - vj * d[j]
            else:
                h = np.zeros(j + 1)
                vj, un = np.zeros(n), np.zeros(n)
            V[:, j], V[:, j + 1] = vj, un
            e = np.linalg.norm(un)                                     # norm
            if e <= 8 * EPS * (j + 2) * np.sqrt(h @ h + e * e):
                e = 0.0
            st["eta"], st["gsave"] = e, g[j]
            st["hp"] = np.zeros(m + 2)
            st["hp"][:j + 1] = h
            col = np.zeros(j + 2)
            col[:j + 1] = h
            column(j, col, e)
            return e, abs(g[j + 1])

        jend = 0
        for j in range(m):
            V[:, j + 1] = A @ Minv(V[:, j])
            hn, est = step(j)
            its += 1
            jend = j + 1
            hist.append(est)
            if hn == 0 or est <= rtol * bn or its >= maxit:
                break
        if keep is not None:
            keep.update(V=V[:, :jend].copy(), Hu=Hu[:jend, :jend - 1].copy(),
                        smax=max(keep.get("smax", 0.0), st.get("smax", 0.0)))
        y = np.zeros(jend)
        for i in range(jend - 1, -1, -1):
            y[i] = (g[i] - R[i, i + 1:jend] @ y[i + 1:]) / R[i, i] if R[i, i] else 0.0
        x = x + Minv(V[:, :jend] @ y)


def _system(n=300, seed=1):
    rng = np.random.default_rng(seed)
    A = 4 * np.eye(n) + 1.5 * rng.standard_normal((n, n)) / np.sqrt(n)
    A[np.arange(n - 1), np.arange(1, n)] -= 1.0
    A[np.arange(1, n), np.arange(n - 1)] -= 1.3
    return A, rng.standard_normal(n)


def _min_residuals(A, Minv, r0, k):
    """min over z in K_i(A M^-1, r0) of |r0 - A M^-1 z|, i = 1..k, by an
    orthonormal basis of the Krylov space and a dense least squares"""
    out, K = [], [r0 / np.linalg.norm(r0)]
    for i in range(1, k + 1):
        K.append(A @ Minv(K[-1]))
        K[-1] /= np.linalg.norm(K[-1])
        Q, _ = np.linalg.qr(np.array(K[:i]).T)
        AQ = A @ np.array([Minv(q) for q in Q.T]).T
        y = np.linalg.lstsq(AQ, r0, rcond=None)[0]
        out.append(np.linalg.norm(r0 - AQ @ y))
    return np.array(out)


def test_residual_estimates_are_the_krylov_minimum():
    A, b = _system()
    d = np.diag(A).copy()
    Minv = lambda v: v / d
    _, hist, _ = lagged_gmres(A, Minv, b, m=12, maxit=12, rtol=0.0)
    ref = _min_residuals(A, Minv, b, 12)
    # the reference orthonormalizes normalized powers, whose conditioning
    # grows with k: it keeps about 1e-10 at k = 12
    np.testing.assert_allclose(hist[1:13], ref, rtol=1e-8)


@pytest.mark.parametrize("m", [5, 30])
def test_restarted_solve_reaches_the_true_residual(m):
    A, b = _system(seed=2)
    d = np.diag(A).copy()
    x, hist, its = lagged_gmres(A, lambda v: v / d, b, m=m, maxit=500, rtol=1e-10)
    assert its < 500
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    assert np.all(np.diff(hist[:m + 1]) <= 1e-12 * hist[0])   # non-increasing in a cycle


def test_arnoldi_relation_when_one_projection_is_not_enough():
    # five dominant eigenvalues and the rest near 1e-7: after five steps each
    # new w lies in span V up to 1e-7 of its norm, one classical projection
    # leaves components of size s ~ eps |w| / eta along V, and only the
    # lagged second projection keeps V orthonormal; A V_k = V_{k+1} H holds
    # for the final columns
    n, m = 400, 14
    rng = np.random.default_rng(4)
    ev = np.concatenate([[1.0, 0.9, 0.8, 0.7, 0.6], 1e-7 * np.linspace(1.0, 2.0, n - 5)])
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = (Q * ev) @ Q.T
    b = rng.standard_normal(n)
    keep = {}
    lagged_gmres(A, lambda v: v, b, m=m, maxit=m, rtol=0.0, keep=keep)
    V, Hu = keep["V"], keep["Hu"]
    k = Hu.shape[1]
    assert k == m - 1 and keep["smax"] > 1e-11
    rel = np.linalg.norm(A @ V[:, :k] - V[:, :k + 1] @ Hu) / np.linalg.norm(Hu)
    assert rel <= 1e-13
    assert np.abs(V[:, :k + 1].T @ V[:, :k + 1] - np.eye(k + 1)).max() <= 1e-13


def test_lucky_breakdowns():
    n = 200
    rng = np.random.default_rng(3)
    e = np.zeros(n)
    e[7] = 1.0
    ident = lambda v: v
    cases = [(4 * np.eye(n), rng.standard_normal(n), 1),                 # A = 4 I
             (np.diag(np.arange(1.0, n + 1)), e, 1),                      # eigenvector
             (np.eye(n) + rng.standard_normal((n, 3)) @ rng.standard_normal((3, n)) / n,
              rng.standard_normal(n), 4)]                                  # I + rank 3
    for A, b, steps in cases:
        x, hist, its = lagged_gmres(A, ident, b, m=30, maxit=100, rtol=1e-12)
        assert its <= steps
        assert np.all(np.isfinite(x))
        assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)
