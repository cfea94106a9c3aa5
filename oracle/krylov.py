"""Restarted GMRES(m) written out (oracle; test infrastructure only).

The paper solves its Newton systems with a matrix-free Krylov method (GMRES;
Section 4.1 and Algorithm 2) without giving restart, orthogonalisation or
stopping details.  This is textbook GMRES (Saad & Schultz): Arnoldi with
modified Gram-Schmidt, Givens rotations on the Hessenberg matrix, x_0 = 0,
stop when the residual estimate |g_{j+1}| <= rtol ||b|| or after ``maxiter``
matrix-vector products, restart every ``restart`` steps.
"""
import numpy as np


def gmres(matvec, b, restart=30, rtol=1e-10, maxiter=300):
    """Solve M x = b.  Returns (x, matvecs_used, final_relative_residual_estimate)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return x, 0, 0.0
    used = 0
    rel = 1.0
    first = True
    while used < maxiter:
        r = b.copy() if first else b - matvec(x)
        first = False
        beta = float(np.linalg.norm(r))
        rel = beta / bnorm
        if beta <= rtol * bnorm:
            break
        m = restart
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gv = np.zeros(m + 1)
        gv[0] = beta
        V[0] = r / beta
        jlast = -1
        for j in range(m):
            w = matvec(V[j])
            used += 1
            for i in range(j + 1):              # modified Gram-Schmidt
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                  # previous rotations on column j
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gv[j + 1] = -sn[j] * gv[j]
            gv[j] = cs[j] * gv[j]
            rel = abs(gv[j + 1]) / bnorm
            jlast = j
            if rel <= rtol or used >= maxiter or breakdown:
                break
        k = jlast + 1
        yk = np.zeros(k)
        for i in range(k - 1, -1, -1):          # back substitution with R = H[:k, :k]
            yk[i] = (gv[i] - np.dot(H[i, i + 1:k], yk[i + 1:k])) / H[i, i]
        x = x + V[:k].T @ yk
        if rel <= rtol:
            break
    return x, used, rel
