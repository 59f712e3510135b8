"""The discrete relativistic lattice Boltzmann update (Sec. II D, Eq. rlb:disc)
with time step delta t' = 1:

    f_i(x + theta_i, t + 1) = f_i(x, t) - (p_i^mu U_mu / (tau p_i^0)) (f_i - f_i^eq)

One step, for every cell x, in the paper's order:
  1. moments N^mu = sum_i f_i p_i^mu and T^{mu nu} = sum_i f_i p_i^mu p_i^nu;
  2. Landau-Lifshitz eigenproblem T^{mu nu} U_nu = eps U^mu (landau.solve);
  3. n = U_mu N^mu, T = eps / (3 n) (equation of state eps = 3 n T), P = eps/3;
  4. relaxation time tau (fixed, or from eta/s, see relaxation_time);
  5. f_i^eq from (n, T, U) (Eq. disc1);
  6. Anderson-Witting relaxation with rate p_i^mu U_mu / (tau p_i^0)
     = (U^0 - theta_i . U / R) / tau;
  7. exact streaming: the post-collision value moves to x + theta_i
     (periodic in every direction).

Arrays: populations f[Q, nz, ny, nx] (x fastest), the same ordering the
library stores on the device.

Solid walls (optional): the paper asks for inversion-paired weights
(w_i = w_inv(i), Sec. II C) so that bounce-back can impose zero velocity on
solid walls.  A solid cell holds no fluid; a population i whose source
cell x - theta_i is solid is replaced by the post-collision population of
the inverse direction at x itself (link-wise bounce-back, stream_with_walls).

Two models share these steps: the third-order model (order 3: 128 points,
R = sqrt(41), J_0..J_29) and the second-order model of Appendix A (order 2:
66 points, R = 3, J_0..J_13, Eq. equi2nd).  They differ in the lattice, the
number of Table I polynomials kept, and the viscosity-tau relation.
"""
import numpy as np

from . import landau
from .equilibrium import Equilibrium, ETA
from .lattice import load_lattice, model_lattice

# shear viscosity eta = n T (tau - 1/2) / (c R): c = 3/2 for the third-order
# model (Sec. III, eta = (2/3) P (tau - 1/2) / R) and c = 7 for the
# second-order model (the numerical fit eta_2nd ~ (1/7) P (tau - 1/2) / R of
# Appendix A); P = n T
VISCOSITY_C = {3: 1.5, 2: 7.0}
KMAX = {3: 30, 2: 14}

FLAG_NONFINITE = 1
FLAG_NONPHYSICAL = 2
FLAG_LANDAU = 4


def moments(lat, f2):
    """f2[Q, C] -> N[C,4], Tm[C,4,4] (step 1)."""
    N = f2.T @ lat.p
    pp = (lat.p[:, :, None] * lat.p[:, None, :]).reshape(lat.Q, 16)
    Tm = (f2.T @ pp).reshape(-1, 4, 4)
    return N, Tm


def macroscopic(lat, f2):
    """Steps 1-3: returns dict with n, eps, T, P, U[C,4] and a status word."""
    N, Tm = moments(lat, f2)
    eps, U, iters, ok = landau.solve(Tm)
    n = np.einsum("ci,ij,cj->c", U, ETA, N)
    T = eps / (3.0 * n)
    flags = 0
    if not np.all(np.isfinite(f2)):
        flags |= FLAG_NONFINITE
    v2 = np.sum(U[:, 1:] ** 2, axis=1) / np.maximum(U[:, 0] ** 2, 1e-300)
    if np.any(~(n > 0)) or np.any(~(eps > 0)) or np.any(~(v2 < 1)):
        flags |= FLAG_NONPHYSICAL
    if not np.all(ok):
        flags |= FLAG_LANDAU
    return dict(N=N, Tm=Tm, n=n, eps=eps, T=T, P=eps / 3.0, U=U, iters=iters, flags=flags)


def relaxation_time(lat, n, T, tau=None, eta_s=None, order=3):
    """Step 4.  Either a fixed tau, or tau from the ratio eta/s per cell:
    the shear viscosity eta = n T (tau - 1/2) / (c R) (VISCOSITY_C, with
    delta t' = 1) and the entropy density s = 4 n - n ln(n / n_eq) with
    n_eq = T^3 in the numerical units of Sec. III (there n = T^3 at rest,
    P = T^4), which give
        tau = 1/2 + (c R / T) (eta/s) (4 - ln(n / T^3)),
    i.e. 1/2 + (3 R / (2 T)) (eta/s) (4 - ln(n / T^3)) for the third-order
    model."""
    if tau is not None:
        return np.full_like(n, float(tau))
    return 0.5 + (VISCOSITY_C[order] * lat.R / T) * eta_s * (4.0 - np.log(n / T**3))


def collide(lat, eq, f2, tau=None, eta_s=None, order=3):
    """Steps 1-6 on f2[Q, C]; returns the post-collision populations and
    the macroscopic state that was used."""
    mac = macroscopic(lat, f2)
    tau_c = relaxation_time(lat, mac["n"], mac["T"], tau, eta_s, order)
    feq = eq(mac["n"], mac["T"], mac["U"]).T                     # [Q, C]
    U = mac["U"]
    # p_i^mu U_mu / p_i^0 = U^0 - (theta_i / R) . U_vec
    rate = (U[:, 0][None, :] - (lat.theta @ U[:, 1:].T) / lat.R) / tau_c[None, :]
    return f2 - rate * (f2 - feq), mac


def stream(lat, f4):
    """Step 7 on f4[Q, nz, ny, nx]: f_new(x + theta_i) = f_post(x)."""
    out = np.empty_like(f4)
    for i in range(lat.Q):
        tx, ty, tz = (int(t) for t in lat.theta[i])
        out[i] = np.roll(f4[i], shift=(tz, ty, tx), axis=(0, 1, 2))
    return out


def stream_with_walls(lat, f4, solid):
    """Step 7 with solid cells solid[nz, ny, nx] (bool): for every fluid
    cell x, f_new_i(x) = f_post_i(x - theta_i) if x - theta_i is fluid,
    else f_post_inv(i)(x) (the population that would have entered the wall
    comes back reversed, on the same shell).  Solid cells hold zeros."""
    out = np.empty_like(f4)
    for i in range(lat.Q):
        tx, ty, tz = (int(t) for t in lat.theta[i])
        moved = np.roll(f4[i], shift=(tz, ty, tx), axis=(0, 1, 2))
        source_solid = np.roll(solid, shift=(tz, ty, tx), axis=(0, 1, 2))     # solid at x - theta_i
        out[i] = np.where(source_solid, f4[lat.inv[i]], moved)
    out[:, solid] = 0.0
    return out


def equilibrium_state(eq, n, eps, vx, vy, vz):
    """Populations at local equilibrium for given n, eps, v (used for
    initial conditions, Sec. III): T = eps / (3 n), U = gamma (1, v)."""
    n = np.asarray(n, np.float64).ravel()
    eps = np.asarray(eps, np.float64).ravel()
    v = np.stack([np.asarray(a, np.float64).ravel() for a in (vx, vy, vz)], axis=1)
    gamma = 1.0 / np.sqrt(1.0 - np.sum(v * v, axis=1))
    U = np.concatenate([gamma[:, None], gamma[:, None] * v], axis=1)
    T = eps / (3.0 * n)
    return eq(n, T, U).T                                         # [Q, C]


class Solver:
    """A periodic nx x ny x nz lattice advanced by Eq. rlb:disc, with the
    third-order (order=3) or the second-order (order=2) model, optionally
    with solid cells (solid: bool array [nz, ny, nx], bounce-back walls)."""

    def __init__(self, nx, ny, nz, tau=None, eta_s=None, lat=None, kmax=None, order=3, solid=None):
        if (tau is None) == (eta_s is None):
            raise ValueError("give exactly one of tau, eta_s")
        if order not in KMAX:
            raise ValueError("order must be 2 or 3")
        self.order = order
        self.lat = lat or model_lattice(order)
        self.eq = Equilibrium(self.lat, KMAX[order] if kmax is None else kmax)
        self.shape = (nz, ny, nx)
        self.C = nx * ny * nz
        self.tau, self.eta_s = tau, eta_s
        self.solid = None
        if solid is not None:
            self.solid = np.asarray(solid, dtype=bool).reshape(self.shape)
            if self.solid.all():
                raise ValueError("no fluid cell")
        self.f = None
        self.t = 0
        self.flags = 0

    def init_fields(self, n, eps, vx, vy, vz):
        f2 = equilibrium_state(self.eq, n, eps, vx, vy, vz)
        self.f = f2.reshape((self.lat.Q,) + self.shape)
        if self.solid is not None:
            self.f[:, self.solid] = 0.0
        self.t = 0

    def _fluid(self):
        return np.ones(self.C, dtype=bool) if self.solid is None else ~self.solid.ravel()

    def step(self, nsteps=1):
        fluid = self._fluid()
        for _ in range(nsteps):
            f2 = self.f.reshape(self.lat.Q, self.C)
            fs = np.zeros_like(f2)
            fs[:, fluid], mac = collide(self.lat, self.eq, f2[:, fluid], self.tau, self.eta_s, self.order)
            self.flags |= mac["flags"]
            fs = fs.reshape(self.f.shape)
            self.f = stream(self.lat, fs) if self.solid is None else stream_with_walls(self.lat, fs, self.solid)
            self.t += 1

    def read_fields(self):
        """n, eps, U[4, C], P of the current (pre-collision) state; zero at
        solid cells."""
        fluid = self._fluid()
        mac = macroscopic(self.lat, self.f.reshape(self.lat.Q, self.C)[:, fluid])
        out = dict(n=np.zeros(self.C), eps=np.zeros(self.C), U=np.zeros((4, self.C)), P=np.zeros(self.C),
                   T=np.zeros(self.C))
        for k in ("n", "eps", "P", "T"):
            out[k][fluid] = mac[k]
        out["U"][:, fluid] = mac["U"].T
        out["flags"] = mac["flags"] | self.flags
        return out

    def conserved(self):
        """Box totals of N^0 and T^{0 nu} (the quantities the collision
        keeps per cell and the streaming keeps globally; with walls, N^0 and
        T^{00} stay and the walls exchange momentum).  Solid cells hold
        zeros, so the sum runs over the fluid."""
        f2 = self.f.reshape(self.lat.Q, self.C)
        tot = f2.sum(axis=1)                                     # per population
        p = self.lat.p
        return np.array([np.dot(tot, p[:, 0])] + [np.dot(tot, p[:, 0] * p[:, mu]) for mu in range(4)])
