"""A second, deliberately naive implementation of one step of Eq. rlb:disc
for tiny lattices: pure-Python loops over cells and populations, LAPACK's
eigen-solver for the Landau-Lifshitz frame and the closed-form equilibria
of Appendix B (Eq. equi3rd for the third-order model, Eq. equi2nd for the
second-order model of Appendix A).  It shares nothing with the oracle
except the lattice table, and exists to pin the oracle on small cases."""
import math

import numpy as np

from appendix_equilibrium import equi2nd, equi3rd

ETA = np.diag([1.0, -1.0, -1.0, -1.0])


def landau_eig(Tm):
    w, V = np.linalg.eig(Tm @ ETA)
    for j in range(4):
        u = V[:, j].real
        nrm = u @ ETA @ u
        if nrm > 0 and abs(w[j].imag) < 1e-12 * abs(w[j].real):
            u = u / math.sqrt(nrm)
            if u[0] < 0:
                u = -u
            return w[j].real, u
    raise RuntimeError("no timelike eigenvector")


def step(lat, f, shape, tau=None, eta_s=None, order=3, solid=None):
    """f[Q][nz][ny][nx] (numpy) -> new array after collide + push.
    solid[z][y][x] (optional): solid cells are skipped and hold zeros; a
    post-collision population pushed into a solid cell is pushed back into
    its own cell as the inverse population (found by searching the table
    for -theta on the same shell).
    eta/s gives tau through eta = (2/3) n T (tau - 1/2) / R (Sec. III) for
    the third-order model and eta = (1/7) n T (tau - 1/2) / R (Appendix A)
    for the second-order one."""
    equi = equi3rd if order == 3 else equi2nd
    # tau - 1/2 = eta / (k n T / R) = (R / (k T)) (eta/s) (s/n)
    k = 2.0 / 3.0 if order == 3 else 1.0 / 7.0
    nz, ny, nx = shape
    Q = lat.Q
    out = np.zeros_like(f)
    def inverse(i):
        for j in range(Q):
            if lat.shell[j] == lat.shell[i] and all(lat.theta[j][k] == -lat.theta[i][k] for k in range(3)):
                return j
        raise RuntimeError("no inverse")
    inv = [inverse(i) for i in range(Q)]
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if solid is not None and solid[z][y][x]:
                    continue
                fc = [f[i, z, y, x] for i in range(Q)]
                N = np.zeros(4)
                Tm = np.zeros((4, 4))
                for i in range(Q):
                    N += fc[i] * lat.p[i]
                    Tm += fc[i] * np.outer(lat.p[i], lat.p[i])
                eps, U = landau_eig(Tm)
                n = U @ ETA @ N
                T = eps / (3 * n)
                if tau is not None:
                    t = tau
                else:
                    t = 0.5 + lat.R / (k * T) * eta_s * (4 - math.log(n / T**3))
                for i in range(Q):
                    feq = equi(n, T, U, lat.p[i], lat.w[i])
                    pU = lat.p[i] @ ETA @ U
                    fs = fc[i] - pU / (t * lat.p[i, 0]) * (fc[i] - feq)
                    tx, ty, tz = (int(a) for a in lat.theta[i])
                    zz, yy, xx = (z + tz) % nz, (y + ty) % ny, (x + tx) % nx
                    if solid is not None and solid[zz][yy][xx]:
                        out[inv[i], z, y, x] = fs
                    else:
                        out[i, zz, yy, xx] = fs
    return out
