"""Float64 oracle of the staggered operators, pressure solves, time steps and
pullbacks on a Cartesian grid stretched along any direction (Sec. 2.5
non-uniform grids, e.g. the tanh grid of eq. tanh-grid; App. B kernels with
non-uniform widths |Delta^a_i| and the interpolation weights of
eq. interp-weights).

TEST INFRASTRUCTURE ONLY (see the package docstring). Not used by the product path.

Grid. ``faces[a]`` holds the N_a + 1 face coordinates along direction a,
strictly increasing. x (and z) are periodic: the face N_a closes the period,
cell N_a - 1 neighbours cell 0. y is periodic too (``ywalls=False``: the
Taylor-Green setting of Sec. 7, uniform and tanh grids), or bounded by no-slip
walls at faces[1][0] and faces[1][N_y] (``ywalls=True``: the channel, with the
ghost rule of the channel oracle ``oracle.walls``: tangential ghost = minus the
first interior value, wall faces of u^y = 0 and not unknowns).

Metrics along a direction (code indices, cell i spans [f_i, f_{i+1}]):
  w_i = f_{i+1} - f_i                 cell (pressure-volume) width
  d_i = (w_i + w_{i+1}) / 2           width of the velocity volume around face i
                                      (the face on the right of cell i), i.e. the
                                      distance of the two centres; periodic:
                                      w_N = w_0; walls: d_{-1} = w_0, d_{N-1} = w_{N-1}
  theta_i = w_i / (w_i + w_{i+1})     mass-flux weight of cell i at face i
                                      (1/2 beyond a wall, where it multiplies zeros)

Operators (App. B, written with these widths):
  divergence  r[I] = sum_a (u^a[I] - u^a[I - e_a]) / w^a_{I_a}
  gradient    (G p)^a[I] = (p[I + e_a] - p[I]) / d^a_{I_a}
  diffusion   eq. diff-kernel: for u^a along b, outer width of the velocity
              volume (d^a along a, w^b across), inner widths between the
              neighbouring points (w^a along a, d^b across)
  convection  phi^a[I] = -sum_b (F^{ab}[I] - F^{ab}[I - e_b]) / W^{ab}[I],
              W^{ab} = d^a (b = a) or w^b (b != a), F^{ab} = A^{ab} B^{ab}:
              the transported component averaged along b with weights 1/2,
              A^{ab}[K] = (u^a[K] + u^a[K + e_b]) / 2, and the transporting one
              interpolated along a as the mass-flux average of the two
              pressure-volume faces it spans,
              B^{ab}[K] = theta^a_{K_a} u^b[K] + (1 - theta^a_{K_a}) u^b[K + e_a]
              (1/2 for b = a). On a uniform grid every weight is 1/2; stretched
              along any direction this keeps convection energy-conserving
              (sum Omega_u u . C(u) = 0 for solenoidal u), the reading taken
              for the ambiguous weights of eq. interp-weights.
Volumes: Omega_p[I] = prod_a w^a_{I_a}; Omega_u^a[I] = d^a_{I_a} prod_{b != a} w^b_{I_b}.

Every linear operator is assembled once as a scipy sparse matrix from these
formulas (each row one output value, each column one input value, the ghost
rule folded into the column coefficients); the convection is a sum of
products of such interpolation matrices. Pullbacks are the transposes of the
same matrices (Sec. 3.4 rule), so no pullback formula is written separately.

Pressure (Sec. 2.6.1): the direct solve is the augmented system
[L e; e^T 0][p; lam] = [r; 0] with L = D G, whose p has zero mean and satisfies
D G p = r - mean_w(r) (mean_w the volume-weighted mean); the iterative solve
is CG on the symmetric A = -Omega_p D G, applied as the chain of scaling,
divergence and gradient.

Arrays: velocity (d, [N_z,] N_y, N_x), pressure ([N_z,] N_y, N_x).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import ins

Y = 1


class StretchedGrid:
    """Metrics and assembled operators of one stretched grid."""

    def __init__(self, faces, ywalls=False):
        self.faces = [np.asarray(f, dtype=np.float64) for f in faces]
        for f in self.faces:
            assert f.ndim == 1 and f.size >= 3 and np.all(np.diff(f) > 0)
        self.d = len(self.faces)
        assert self.d in (2, 3)
        self.n = tuple(f.size - 1 for f in self.faces)
        self.ywalls = bool(ywalls)
        self.shape = tuple(reversed(self.n))  # array shape of a pressure field
        self.ncell = int(np.prod(self.n))
        self.w = [np.diff(f) for f in self.faces]
        # cell coordinates of every flat cell index (C order over (z, y, x))
        grids = np.meshgrid(*[np.arange(m) for m in self.shape], indexing="ij")
        self.I = [grids[self.d - 1 - a].ravel() for a in range(self.d)]
        self._assemble()

    # ------------------------------------------------------------ metrics
    def periodic(self, a):
        return not (a == Y and self.ywalls)

    def width(self, a, i):
        """w^a_i; periodic wrap, or the mirrored row beyond a wall."""
        n = self.n[a]
        i = np.asarray(i)
        if self.periodic(a):
            return self.w[a][np.mod(i, n)]
        return self.w[a][np.clip(i, 0, n - 1)]

    def dist(self, a, i):
        """d^a_i, the velocity-volume width around face i (i = -1 .. N - 1)."""
        n = self.n[a]
        i = np.asarray(i)
        if self.periodic(a):
            j = np.mod(i, n)
            return 0.5 * (self.w[a][j] + self.w[a][np.mod(j + 1, n)])
        out = 0.5 * (self.width(a, i) + self.width(a, i + 1))
        return np.where((i <= -1) | (i >= n - 1), self.width(a, i), out)

    def theta(self, a, i):
        """Mass-flux weight of cell i at face i along a."""
        n = self.n[a]
        i = np.asarray(i)
        t = self.width(a, i) / (self.width(a, i) + self.width(a, i + 1))
        if self.periodic(a):
            return t
        return np.where((i < 0) | (i >= n - 1), 0.5, t)

    def volumes_p(self):
        v = np.ones(self.ncell)
        for a in range(self.d):
            v = v * self.w[a][self.I[a]]
        return v.reshape(self.shape)

    def volumes_u(self):
        out = np.ones((self.d, self.ncell))
        for a in range(self.d):
            for b in range(self.d):
                out[a] *= self.dist(a, self.I[a]) if b == a else self.w[b][self.I[b]]
        return out.reshape((self.d,) + self.shape)

    def dof_mask(self):
        """1 on the velocity unknowns; 0 on the stored upper-wall face of u^y (walls)."""
        m = np.ones((self.d, self.ncell))
        if self.ywalls:
            m[Y, self.I[Y] == self.n[Y] - 1] = 0.0
        return m.reshape((self.d,) + self.shape)

    # ------------------------------------------------------------ indexing
    def _cell(self, J):
        """Flat pressure index of cell J (periodic wrap; J_y in range for walls)."""
        k = np.zeros_like(J[0])
        for a in reversed(range(self.d)):
            k = k * self.n[a] + (np.mod(J[a], self.n[a]) if self.periodic(a) else J[a])
        return k

    def _vel(self, c, J):
        """(columns, coefficients) of u^c[J] for cells J one beyond the grid at most,
        the ghost rule of a wall applied."""
        J = [np.asarray(j).copy() for j in J]
        coef = np.ones(J[0].shape)
        if self.ywalls:
            ny = self.n[Y]
            r = J[Y]
            if c == Y:
                coef = np.where((r >= 0) & (r <= ny - 2), 1.0, 0.0)
                J[Y] = np.clip(r, 0, ny - 1)
            else:
                coef = np.where((r < 0) | (r > ny - 1), -1.0, 1.0)
                J[Y] = np.clip(r, 0, ny - 1)
        return c * self.ncell + self._cell(J), coef

    def _shift(self, J, a, s):
        K = [j.copy() for j in J]
        K[a] = K[a] + s
        return K

    # ------------------------------------------------------------ assembly
    def _mat(self, rows, cols, vals, shape):
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=shape)

    def _interp(self, c, J0, w0, J1, w1):
        """Rows = cells: w0 u^c[J0] + w1 u^c[J1] (one row per flat cell index)."""
        rows, cols, vals = [], [], []
        idx = np.arange(self.ncell)
        for J, w in ((J0, w0), (J1, w1)):
            col, cf = self._vel(c, J)
            rows.append(idx)
            cols.append(col)
            vals.append(cf * w)
        return self._mat(rows, cols, vals, (self.ncell, self.d * self.ncell))

    def _assemble(self):
        d, nc = self.d, self.ncell
        I = self.I
        idx = np.arange(nc)
        # divergence (App. B eq. div-kernel)
        rows, cols, vals = [], [], []
        for a in range(d):
            iw = 1.0 / self.w[a][I[a]]
            for s, sg in ((0, 1.0), (-1, -1.0)):
                col, cf = self._vel(a, self._shift(I, a, s))
                rows.append(idx)
                cols.append(col)
                vals.append(sg * cf * iw)
        self.D = self._mat(rows, cols, vals, (nc, d * nc))
        # gradient (eq. presgrad-kernel), interior faces only
        rows, cols, vals = [], [], []
        for a in range(d):
            ok = np.ones(nc, dtype=bool)
            if a == Y and self.ywalls:
                ok = I[Y] <= self.n[Y] - 2
            idd = 1.0 / self.dist(a, I[a])
            for s, sg in ((1, 1.0), (0, -1.0)):
                rows.append((a * nc + idx)[ok])
                cols.append(self._cell(self._shift(I, a, s))[ok])  # rows beyond a wall are filtered out
                vals.append((sg * idd)[ok])
        self.G = self._mat(rows, cols, vals, (d * nc, nc))
        self.M = sp.diags(self.dof_mask().ravel())
        # diffusion (eq. diff-kernel), with ghosts
        rows, cols, vals = [], [], []
        for a in range(d):
            for b in range(d):
                if b == a:
                    o = 1.0 / self.dist(a, I[a])
                    ir = 1.0 / self.width(a, I[a] + 1)
                    il = 1.0 / self.width(a, I[a])
                else:
                    o = 1.0 / self.w[b][I[b]]
                    ir = 1.0 / self.dist(b, I[b])
                    il = 1.0 / self.dist(b, I[b] - 1)
                for s, wgt in ((1, o * ir), (0, -o * (ir + il)), (-1, o * il)):
                    col, cf = self._vel(a, self._shift(I, b, s))
                    rows.append(a * nc + idx)
                    cols.append(col)
                    vals.append(cf * wgt)
        self.K = self.M @ self._mat(rows, cols, vals, (d * nc, d * nc))
        # convection: per (a, b) the factors at K = I and K = I - e_b and the scaling
        self.conv_terms = []
        for a in range(d):
            for b in range(d):
                W = self.dist(a, I[a]) if b == a else self.w[b][I[b]]
                for sh in (0, -1):
                    Kc = self._shift(I, b, sh)
                    A = self._interp(a, Kc, 0.5, self._shift(Kc, b, 1), 0.5)
                    th = np.full(nc, 0.5) if b == a else self.theta(a, Kc[a])
                    B = self._interp(b, Kc, th, self._shift(Kc, a, 1), 1.0 - th)
                    sgn = -1.0 if sh == 0 else 1.0
                    S = self.M @ sp.csr_matrix((sgn / W, (a * nc + idx, idx)), shape=(d * nc, nc))
                    self.conv_terms.append((A, B, S))
        self.L = (self.D @ self.G).tocsc()
        e = sp.csr_matrix(np.ones((nc, 1)))
        self.aug = sp.bmat([[self.L, e], [e.T, None]], format="csc")
        self._lu = None
        self._luT = None

    # ------------------------------------------------------------ forward
    def _v(self, u):
        return np.asarray(u, dtype=np.float64).reshape(-1)

    def _vel_out(self, x):
        return x.reshape((self.d,) + self.shape)

    def divergence(self, u):
        return (self.D @ self._v(u)).reshape(self.shape)

    def gradient(self, p):
        return self._vel_out(self.G @ self._v(p))

    def diffusion(self, u, nu):
        return self._vel_out(nu * (self.K @ self._v(u)))

    def convection(self, u):
        x = self._v(u)
        out = np.zeros(self.d * self.ncell)
        for A, B, S in self.conv_terms:
            out += S @ ((A @ x) * (B @ x))
        return self._vel_out(out)

    def rhs(self, u, nu, force=None):
        """F(u) = C(u) + nu diffusion (+ a constant force on the unknowns)."""
        out = self.convection(u) + self.diffusion(u, nu)
        if force is not None:
            m = self.dof_mask()
            for a in range(self.d):
                out[a] += float(force[a]) * m[a]
        return out

    def laplacian(self, p):
        return (self.L @ self._v(p)).reshape(self.shape)

    def poisson_solve(self, r):
        """Direct solver of Sec. 2.6.1 (augmented system, sparse LU)."""
        if self._lu is None:
            self._lu = spla.splu(self.aug)
        sol = self._lu.solve(np.concatenate([self._v(r), [0.0]]))
        return sol[: self.ncell].reshape(self.shape)

    def cg_solve(self, r, rtol=1e-12, maxiter=20000):
        """Iterative solver of Sec. 2.6.1: CG on A = -Omega_p D G for
        A p = Omega_p (mean_w(r) - r) from p = 0; stops at ||res|| <= rtol ||res_0||
        or after maxiter iterations (or when p . A p <= 0). Returns (p, iterations, relres)."""
        om = self.volumes_p().ravel()
        rv = self._v(r)
        b = om * (np.sum(om * rv) / np.sum(om) - rv)
        x = np.zeros_like(b)
        res = b.copy()
        dv = res.copy()
        rr = rr0 = float(res @ res)
        it = 0
        if rr0 == 0.0:
            return x.reshape(self.shape), 0, 0.0
        while it < maxiter and rr > rtol * rtol * rr0:
            q = -om * (self.L @ dv)
            pq = float(dv @ q)
            if not pq > 0.0:
                rr = 0.0
                break
            alpha = rr / pq
            x = x + alpha * dv
            res = res - alpha * q
            rr_new = float(res @ res)
            dv = res + (rr_new / rr) * dv
            rr = rr_new
            it += 1
        return x.reshape(self.shape), it, float(np.sqrt(rr / rr0))

    def project(self, u):
        """P u = u - G L^{-1} D u on the unknowns (Sec. 2.6.2); returns (P u, p)."""
        p = self.poisson_solve(self.divergence(u))
        return self._vel_out(self.M @ (self._v(u) - self.G @ self._v(p))), p

    # ------------------------------------------------------------ pullbacks
    def divergence_vjp(self, rbar):
        return self._vel_out(self.M @ (self.D.T @ self._v(rbar)))

    def gradient_vjp(self, gbar):
        return (self.G.T @ (self.M @ self._v(gbar))).reshape(self.shape)

    def diffusion_vjp(self, fbar, nu):
        return self._vel_out(nu * (self.M @ (self.K.T @ self._v(fbar))))

    def convection_vjp(self, u, fbar):
        """Transpose of ``convection`` at u, term by term: y = S (A u * B u) gives
        ubar = A^T (S^T ybar * B u) + B^T (S^T ybar * A u)."""
        x = self._v(u)
        fb = self._v(fbar)
        out = np.zeros_like(x)
        for A, B, S in self.conv_terms:
            g = S.T @ fb
            out += A.T @ (g * (B @ x)) + B.T @ (g * (A @ x))
        return self._vel_out(self.M @ out)

    def rhs_vjp(self, u, fbar, nu):
        return self.convection_vjp(u, fbar) + self.diffusion_vjp(fbar, nu)

    def poisson_solve_vjp(self, pbar):
        """Transpose of the direct solve: the first block of aug^{-T} [pbar; 0]."""
        if self._luT is None:
            self._luT = spla.splu(self.aug.T.tocsc())
        sol = self._luT.solve(np.concatenate([self._v(pbar), [0.0]]))
        return sol[: self.ncell].reshape(self.shape)

    def project_vjp(self, ubar_out):
        """P^T v = v - D^T L^{-T} G^T v on the unknowns."""
        v = self._vel_out(self.M @ self._v(ubar_out))
        return v - self.divergence_vjp(self.poisson_solve_vjp(self.gradient_vjp(v)))

    # ------------------------------------------------------------ steps
    def _fns(self, nu, force=None):
        return dict(rhs_fn=lambda v: self.rhs(v, nu, force), project_fn=lambda v: self.project(v)[0])

    def step_rk4(self, u0, nu, dt, force=None):
        return ins.step_rk4(u0, None, nu, dt, **self._fns(nu, force))

    def step_wray3(self, u0, nu, dt, force=None):
        return ins.step_wray3(u0, None, nu, dt, **self._fns(nu, force))

    def step_rk4_vjp(self, u0, u1bar, nu, dt, force=None):
        return ins.step_rk4_vjp(u0, u1bar, None, nu, dt, rhs_vjp_fn=lambda v, fb: self.rhs_vjp(v, fb, nu),
                                project_vjp_fn=self.project_vjp, **self._fns(nu, force))

    def step_wray3_vjp(self, u0, u1bar, nu, dt, force=None):
        return ins.step_wray3_vjp(u0, u1bar, None, nu, dt, rhs_vjp_fn=lambda v, fb: self.rhs_vjp(v, fb, nu),
                                  project_vjp_fn=self.project_vjp, **self._fns(nu, force))
