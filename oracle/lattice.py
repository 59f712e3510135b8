"""Discrete 4-momenta and weights (Sec. II C: Eqs. dio, mrecon, mrecon2).

A lattice point i carries an integer spatial displacement theta_i with
|theta_i|^2 = R^2, an energy p0_i (a zero of the radial polynomial) and a
weight w_i.  Its 4-momentum is p_i = p0_i (1, theta_i / R) (Eq. mrecon).

The weights themselves sit in the paper's supplement; the tables read here
were recomputed from the paper's conditions (Eqs. eqs:eqs, and the same
conditions up to second order for the model of Appendix A) and are checked
against them by the tests.  This module has its own parser and shares no
code with the library.
"""
import os
import numpy as np

ORACLE_DIR = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(ORACLE_DIR)


def default_table_path(name="d3q128"):
    return os.path.join(REPO, "paper_1301_3423_amd", "lattice", name + ".txt")


class Lattice:
    """theta[Q,3] (int), p0[Q], w[Q], shell[Q], inv[Q] and the 4-momenta
    p[Q,4] = p0 (1, theta/R)."""

    def __init__(self, theta, shell, p0, w, r2):
        self.theta = np.asarray(theta, dtype=np.int64)
        self.shell = np.asarray(shell, dtype=np.int64)
        self.p0 = np.asarray(p0, dtype=np.float64)
        self.w = np.asarray(w, dtype=np.float64)
        self.Q = len(self.w)
        self.R2 = int(r2)
        self.R = float(np.sqrt(r2))
        # Eq. mrecon: p^mu = p0 (1, theta / R)
        self.p = np.empty((self.Q, 4))
        self.p[:, 0] = self.p0
        self.p[:, 1:] = self.p0[:, None] * self.theta / self.R
        # spatial inverse of each point (same energy, opposite theta)
        key = {(int(s), tuple(t)): i for i, (s, t) in enumerate(zip(self.shell, self.theta))}
        self.inv = np.array([key[(int(s), tuple(-t))] for s, t in zip(self.shell, self.theta)])


def model_lattice(order=3):
    """The lattice of the third-order model (order 3: d3q128, R^2 = 41) or
    of the second-order model of Appendix A (order 2: d3q66, R^2 = 9)."""
    return load_lattice(default_table_path({3: "d3q128", 2: "d3q66"}[order]))


def load_lattice(path=None):
    path = path or default_table_path()
    rows = []
    r2 = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                if "R^2 =" in line:
                    r2 = int(line.split("R^2 =")[1].split(",")[0])
                continue
            if not line.strip():
                continue
            tok = line.split()
            rows.append((int(tok[2]), int(tok[3]), int(tok[4]), int(tok[5]),
                         float.fromhex(tok[6]), float.fromhex(tok[7])))
    shell = [r[0] for r in rows]
    theta = [r[1:4] for r in rows]
    p0 = [r[4] for r in rows]
    w = [r[5] for r in rows]
    return Lattice(theta, shell, p0, w, r2)
