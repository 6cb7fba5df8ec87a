"""FP64 CPU oracle of one time step of the segregated predictor multi-corrector -- TEST
INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this module; the GPU library never calls it and shares no code with it.

What it computes (Sec. 3.4 and Sec. 3.5, for the linear(ised) unified continuum on a fixed mesh):

* the semi-discrete balance equations R(y_dot, y, u_s) = K_rate (y_dot - (f, 0)) + K_state y +
  K_disp (u_s, 0) = 0 with y = (v, p) per block row, and the kinematic equation of the solid
  R_k = u_dot_s - v = 0 on the velocity rows that a solid element touches;
* the first-order generalized-alpha method: the equations are collocated at y_dot(alpha_m) and
  y(alpha_f), and y_{n+1} = y_n + dt y_dot_n + gamma dt (y_dot_{n+1} - y_dot_n) for every field
  (v, p, the solid displacement u_s and the mesh displacement u_hat, whose rate is the mesh
  velocity v_hat);
* the predictor (same-Y: y_{n+1} = y_n, y_dot_{n+1} = (gamma - 1)/gamma y_dot_n) and the
  multi-corrector: the solid displacement update by the segregated kinematic increment, the mesh
  motion by harmonic extension with the solid displacement as its Dirichlet data on solid nodes
  and zero on the other Dirichlet nodes, the mesh velocity from the mesh displacement, the
  residual of the balance equations at the intermediate states, the stopping test against the
  residual of the first corrector, and the corrector system tangent dy_dot = -R / (alpha_f gamma
  dt) solved exactly (sparse LU), followed by the rate and state updates of (v, p).

Readings (the paper leaves them open): the velocity-rate increment used by the solid update of a
corrector is the one computed by the previous corrector (zero in the first), with the kinematic
residual taken at the iterate before that increment was applied, so the kinematic equation holds
after every solid update; the reference residual of the relative stopping test is that of the
first corrector; steps 5 and 6 (flow rates and reduced outlet models) are absent.

Pinned in ``tests/test_corrector_oracle.py``: against a monolithic solve of the generalized-alpha
equations written directly from their definition; second-order convergence and exact energy
conservation (rho_inf = 1) on an oscillator and a decaying mode with known solutions; the kinematic
residual vanishing after convergence; constant Dirichlet data extended as a constant.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import assembly as asm


def scalar_csr(rp, ci, val) -> sp.csr_matrix:
    """The (nb*bs) x (nb*bs) scalar matrix of a block-CSR pattern with (nnzb, bs, bs) values."""
    val = np.asarray(val)
    if val.ndim == 1:
        val = val.reshape(-1, 1, 1)
    nb = len(rp) - 1
    return sp.bsr_matrix((val, np.asarray(ci), np.asarray(rp)), shape=(nb * val.shape[1], nb * val.shape[2])).tocsr()


def assembled_operators(s, prm: dict):
    """dt -> {form: scalar CSR matrix} for the four forms of oracle.assembly on a generated system
    (tets, pattern, Dirichlet mask), at rest."""
    def at(dt):
        q = dict(prm)
        q["dt"] = dt
        return {f: scalar_csr(s.rp, s.ci, asm.tangent(s.tv, s.tp, s.tsolid, s.xyz, s.rp, s.ci, s.mask, q, form=f))
                for f in asm.FORMS}
    return at


def solid_rows_of(s) -> np.ndarray:
    """Block rows whose velocity a solid element uses (uint8, 1 = solid)."""
    out = np.zeros(s.n_b, np.uint8)
    out[np.asarray(s.tv)[np.asarray(s.tsolid).astype(bool)].reshape(-1)] = 1
    return out


def harmonic_extension(L: sp.csr_matrix, dirichlet: np.ndarray, uD: np.ndarray) -> np.ndarray:
    """The discrete Laplace equation of the mesh motion: L_FF u_F = -L_FD u_D on the free nodes,
    u = u_D on the Dirichlet nodes.  L: unreduced n x n; uD: (n, 3), read on Dirichlet nodes."""
    d = np.asarray(dirichlet).astype(bool)
    f = ~d
    out = np.where(d[:, None], uD, 0.0)
    if f.any():
        L = L.tocsr()
        LFF = L[f][:, f].tocsc()
        LFD = L[f][:, d]
        out[f] = spla.splu(LFF).solve(-(LFD @ uD[d]))
    return out


class Stepper:
    """State and time step of the predictor multi-corrector.

    operators: dt -> {"tangent", "rate", "state", "disp"}: scalar 4nb x 4nb matrices (the tangent
    with unit Dirichlet diagonal, the residual parts with zero Dirichlet rows and columns).
    solid: (nb,) rows with a kinematic equation.  L: unreduced mesh Laplacian (nL x nL);
    mesh_dirichlet: (nL,) flags; blk_of_phys: (nL,) block row of each mesh node."""

    def __init__(self, operators, solid, L, mesh_dirichlet, blk_of_phys, rho_inf: float, dt0: float,
                 tol_R: float = 1e-6, tol_A: float = 1e-14, max_correctors: int = 10):
        self.operators = operators
        self.solid = np.asarray(solid).astype(bool)
        self.L = sp.csr_matrix(L)
        self.mdir = np.asarray(mesh_dirichlet).astype(bool)
        self.bop = np.asarray(blk_of_phys)
        self.am, self.af, self.gamma = asm.genalpha(rho_inf)
        self.tol_R, self.tol_A, self.max_correctors = tol_R, tol_A, max_correctors
        nb = self.solid.size
        nL = self.bop.size
        self.nb, self.nL = nb, nL
        # state at t_n: (v, p) and rates per block row; solid displacement and rate; mesh
        # displacement and velocity per mesh node
        self.y = np.zeros((nb, 4)); self.yd = np.zeros((nb, 4))
        self.us = np.zeros((nb, 3)); self.usd = np.zeros((nb, 3))
        self.mu = np.zeros((nL, 3)); self.mv = np.zeros((nL, 3))
        self._set_dt(dt0)

    def _set_dt(self, dt):
        self.dt = dt
        self.K = self.operators(dt)
        self.lu = spla.splu(sp.csc_matrix(self.K["tangent"]))

    def residual(self, yd_am, y_af, us_af, f):
        """R(y_dot(alpha_m), y(alpha_f), u_s(alpha_f)) of the balance equations (4 nb)."""
        w = yd_am.copy()
        if f is not None:
            w[:, :3] -= f
        u4 = np.zeros_like(y_af)
        u4[:, :3] = us_af
        return self.K["rate"] @ w.reshape(-1) + self.K["state"] @ y_af.reshape(-1) + self.K["disp"] @ u4.reshape(-1)

    def kinematic_residual(self, usd_am, y_af):
        """R_k = u_dot_s(alpha_m) - v(alpha_f) on the solid rows, zero elsewhere."""
        return np.where(self.solid[:, None], usd_am - y_af[:, :3], 0.0)

    def step(self, dt: float, f=None) -> dict:
        """Advance the state by dt under the body force f ((nb, 3) or None).  Returns the corrector
        count, the first and last residual norms, the summed mesh and linear iterations (0 here:
        direct solves) and whether the stopping test held."""
        stats = dict(correctors=0, converged=False, res0=0.0, res=0.0, resetups=0)
        if dt != self.dt:
            self._set_dt(dt)
            stats["resetups"] = 1
        am, af, g = self.am, self.af, self.gamma
        c = (g - 1.0) / g
        # predictor
        y1, yd1 = self.y.copy(), c * self.yd
        us1, usd1 = self.us.copy(), c * self.usd
        mu1, mv1 = self.mu.copy(), c * self.mv
        y_af = self.y + af * (y1 - self.y)
        Rk = self.kinematic_residual(self.usd + am * (usd1 - self.usd), y_af)
        dvd = np.zeros((self.nb, 3))
        res0 = None
        for l in range(1, self.max_correctors + 1):
            stats["correctors"] = l
            # steps 1-2: solid displacement
            dusd = (af * g * dt / am) * dvd - Rk / am
            dusd[~self.solid] = 0.0
            usd1 = usd1 + dusd
            us1 = us1 + g * dt * dusd
            y_af = self.y + af * (y1 - self.y)
            Rk = self.kinematic_residual(self.usd + am * (usd1 - self.usd), y_af)
            # steps 3-4: mesh motion and mesh velocity
            uD = np.where((self.mdir & self.solid[self.bop])[:, None], us1[self.bop], 0.0)
            mu1 = harmonic_extension(self.L, self.mdir, uD)
            mv1 = (mu1 - self.mu) / (g * dt) + c * self.mv
            # step 7: residual at the intermediate states
            yd_am = self.yd + am * (yd1 - self.yd)
            us_af = self.us + af * (us1 - self.us)
            R = self.residual(yd_am, y_af, us_af, f)
            # step 8: stopping test
            res = float(np.linalg.norm(R))
            if res0 is None:
                res0 = res
            stats["res0"], stats["res"] = res0, res
            if (res0 > 0.0 and res / res0 <= self.tol_R) or res <= self.tol_A:
                stats["converged"] = True
                break
            if l == self.max_correctors:
                break
            # step 9: corrector system
            d = self.lu.solve(-R / (af * g * dt)).reshape(self.nb, 4)
            # step 10: updates of (v, p) and their rates
            yd1 = yd1 + d
            y1 = y1 + g * dt * d
            dvd = np.where(self.solid[:, None], d[:, :3], 0.0)
        self.y, self.yd, self.us, self.usd, self.mu, self.mv = y1, yd1, us1, usd1, mu1, mv1
        return stats
