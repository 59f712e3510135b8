"""Landau-Lifshitz frame: the eigenproblem T^{alpha beta} U_beta = eps U^alpha
(Eq. eigenproblem, and its discrete use after Eq. rlb:disc).

Method (oracle's choice, deliberately plain): shifted power iteration on
the mixed tensor T^mu_nu = T^{mu alpha} eta_{alpha nu}, whose timelike
eigenvector is U with eigenvalue eps and whose spacelike eigenvalues are
minus the principal pressures.  With the shift sigma = eps0/2 the timelike
eigenvalue dominates by a factor >= 3 whenever the principal pressures lie
in [0, eps].  Iterates are normalised in the Euclidean norm; the converged
vector is normalised to U.U = 1 with U^0 > 0.

Start: the exact solution for an ideal fluid with P = eps/3, written in
terms of E = T^00 and |M| = |T^{0i}|: v0 = 3x / (2 + sqrt(4 - 3x^2)) along
M with x = |M|/E, and eps0 = E - |M| v0.
"""
import numpy as np

ETA = np.diag([1.0, -1.0, -1.0, -1.0])
MAX_ITER = 400


def solve(Tmn):
    """Tmn[c,4,4] (contravariant) -> eps[c], U[c,4], iterations[c],
    converged[c] (bool)."""
    Tmn = np.asarray(Tmn, dtype=np.float64)
    c = Tmn.shape[0]
    E = Tmn[:, 0, 0]
    M = Tmn[:, 0, 1:]
    Mabs = np.sqrt(np.sum(M * M, axis=1))
    x = Mabs / E
    v0 = 3.0 * x / (2.0 + np.sqrt(np.maximum(4.0 - 3.0 * x * x, 0.0)))
    dirn = np.where(Mabs[:, None] > 0, M / np.where(Mabs > 0, Mabs, 1.0)[:, None], 0.0)
    v = v0[:, None] * dirn
    eps0 = E - Mabs * v0
    sigma = 0.5 * eps0
    # mixed tensor T^mu_nu = T^{mu a} eta_{a nu}, shifted
    A = Tmn @ ETA + sigma[:, None, None] * np.eye(4)[None]
    u = np.concatenate([np.ones((c, 1)), v], axis=1)
    u /= np.linalg.norm(u, axis=1)[:, None]
    iters = np.zeros(c, dtype=np.int64)
    done = np.zeros(c, dtype=bool)
    tol = 4.0 * np.finfo(np.float64).eps
    for it in range(MAX_ITER):
        act = ~done
        if not act.any():
            break
        ua = u[act]
        un = np.einsum("cij,cj->ci", A[act], ua)
        un /= np.linalg.norm(un, axis=1)[:, None]
        change = np.max(np.abs(un - ua), axis=1)
        u[act] = un
        iters[act] += 1
        newly = change <= tol
        idx = np.nonzero(act)[0]
        done[idx[newly]] = True
    # normalise to U.U = 1, U^0 > 0
    norm2 = u[:, 0] ** 2 - np.sum(u[:, 1:] ** 2, axis=1)
    ok = (norm2 > 0) & done
    s = np.sign(u[:, 0])
    U = u * (s / np.sqrt(np.where(norm2 > 0, norm2, 1.0)))[:, None]
    U_low = U @ ETA
    eps = np.einsum("ci,cij,cj->c", U_low, Tmn, U_low)
    return eps, U, iters, ok
