"""Right-preconditioned Krylov drivers (oracle; test infrastructure).

What this follows
-----------------
Sec. IV-A (System setup, Workloads): BiCGSTAB with standard parameters and
GMRES with restart k = 30, stopping when ||b - A x_k|| / ||b - A x_0|| drops
below the tolerance; Table III gives the per-iteration work (BiCGSTAB: 2
preconditioner applies, 2 SpMV; GMRES: 1 and 1 plus the orthogonalisation).

Readings
--------
* Right preconditioning (A M^{-1} y = b, x = M^{-1} y), so the monitored
  residual is the residual of the original system.  GMRES is the flexible
  variant (FGMRES, Saad 1993), which stores the preconditioned vectors Z and
  so stays correct when M^{-1} changes between iterations (reduced precision,
  learned correction).
* BiCGSTAB is van der Vorst's 1992 algorithm, with the stopping test on the
  residual r at the end of each full step (no exit half-way on s: since
  omega minimises ||s - omega t||, ||r|| <= ||s|| and the step count is the
  same).  When the recursive residual meets the tolerance the true residual
  b - A x is recomputed; if it does not meet it, the iteration restarts from
  the true residual.
* Arnoldi uses classical Gram-Schmidt; a second CGS pass runs when the norm
  of w drops by more than a factor 10 in the first pass.
* One iteration = one preconditioner apply + one SpMV for FGMRES, two of
  each for BiCGSTAB (Table III).

A, M are callables on NumPy arrays of any fixed shape; dots are over all
entries in FP64.
"""
import numpy as np

REORTH_RATIO = 0.1


def _dot(a, b):
    return float(np.dot(a.ravel(), b.ravel()))


def _nrm(a):
    return float(np.sqrt(_dot(a, a)))


def bicgstab(A, b, M=None, x0=None, tol=1e-8, maxiter=1000):
    """Returns (x, info) with info = dict(iterations, converged, history, rel_true)."""
    M = M if M is not None else (lambda v: v.copy())
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    r = b - A(x)
    r0 = _nrm(r)
    hist = [1.0]
    info = dict(iterations=0, converged=r0 == 0.0, history=hist, breakdown=False)
    if r0 == 0.0:
        info["rel_true"] = 0.0
        return x, info
    it = 0
    while it < maxiter:
        rhat = r.copy()
        rho_old = alpha = omega = 1.0
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        restart = False
        while it < maxiter:
            rho = _dot(rhat, r)
            if rho == 0.0 or not np.isfinite(rho):
                info["breakdown"] = True
                break
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
            phat = M(p)
            v = A(phat)
            alpha = rho / _dot(rhat, v)
            s = r - alpha * v
            it += 1
            shat = M(s)
            t = A(shat)
            tt = _dot(t, t)
            omega = _dot(t, s) / tt if tt > 0 else 0.0
            x = x + alpha * phat + omega * shat
            r = s - omega * t
            rnorm = _nrm(r)
            hist.append(rnorm / r0)
            if not np.isfinite(rnorm):
                info["breakdown"] = True
                break
            if rnorm <= tol * r0:
                restart = True
                break
            if omega == 0.0:
                info["breakdown"] = True
                break
            rho_old = rho
        r = b - A(x)
        rel = _nrm(r) / r0
        if rel <= tol:
            info["converged"] = True
            break
        if info["breakdown"] or not restart:
            break
    info["iterations"] = it
    info["rel_true"] = _nrm(b - A(x)) / r0
    return x, info


def fgmres(A, b, M=None, x0=None, tol=1e-8, restart=30, maxiter=1000, capture=None):
    """Flexible GMRES(restart).  Returns (x, info).

    `capture`, if given, is called with each iterate x_k after every
    iteration (used to generate training pairs); it costs one extra
    small solve per iteration.
    """
    M = M if M is not None else (lambda v: v.copy())
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    r = b - A(x)
    beta = _nrm(r)
    r0 = beta
    hist = [1.0]
    info = dict(iterations=0, converged=r0 == 0.0, history=hist, reorth=0)
    if r0 == 0.0:
        info["rel_true"] = 0.0
        return x, info
    it = 0
    m = restart
    while it < maxiter:
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        ncols = 0
        for j in range(m):
            Z.append(M(V[j]))
            w = A(Z[j])
            wn0 = _nrm(w)
            h = np.array([_dot(V[i], w) for i in range(j + 1)])
            w = w - sum(h[i] * V[i] for i in range(j + 1))
            hn = _nrm(w)
            if hn < REORTH_RATIO * wn0:
                h2 = np.array([_dot(V[i], w) for i in range(j + 1)])
                w = w - sum(h2[i] * V[i] for i in range(j + 1))
                h = h + h2
                hn = _nrm(w)
                info["reorth"] += 1
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):                    # previous Givens rotations
                a, bb = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * bb
                H[i + 1, j] = -sn[i] * a + cs[i] * bb
            a, bb = H[j, j], H[j + 1, j]
            den = np.hypot(a, bb)
            cs[j], sn[j] = (1.0, 0.0) if den == 0 else (a / den, bb / den)
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            ncols = j + 1
            hist.append(abs(g[j + 1]) / r0)
            if capture is not None:
                y = np.linalg.solve(np.triu(H[:ncols, :ncols]), g[:ncols])
                capture(x + sum(y[i] * Z[i] for i in range(ncols)))
            if hn == 0.0 or abs(g[j + 1]) <= tol * r0 or it >= maxiter:
                break
            V.append(w / hn)
        y = np.linalg.solve(np.triu(H[:ncols, :ncols]), g[:ncols])
        x = x + sum(y[i] * Z[i] for i in range(ncols))
        r = b - A(x)
        beta = _nrm(r)
        if beta <= tol * r0:
            info["converged"] = True
            break
        if not np.isfinite(beta):
            break
    info["iterations"] = it
    info["rel_true"] = _nrm(b - A(x)) / r0
    return x, info
