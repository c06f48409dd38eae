"""A stack of spherical shells: Cartesian gradient, boundaries, SSP-RK3 -- oracle side.

Test infrastructure only (see package docstring).

Data layout (shared with the GPU path's C interface, so that arrays can be
compared element by element): shells are concatenated in the given order
(grouped by instance, inner to outer); each shell holds a block
[component][r][theta][phi] with N_r*S points, S = (L+1) * 2(L+1).

Per-point inputs beside the 50 fields: H [4] (gauge source H_a), dH [16]
(d_a H_b, row a*4+b, a = 0 is the time derivative), u_bg [50] (the background
state that freezes the characteristic projections at interfaces).
"""

import numpy as np

from . import grid as _grid
from . import spectral as _spec
from . import dp5 as _dp5
from . import gh as _gh
from . import tensor_filter as _tf


class Shell:
    def __init__(self, instance, n_r, L, r_in, r_out):
        self.instance = int(instance)
        self.n_r, self.L = int(n_r), int(L)
        self.r_in, self.r_out = float(r_in), float(r_out)


class Domain:
    """Shells of one or more independent instances (black holes)."""

    def __init__(self, shells, filter_params=None, filter_kind=1, interface_from_state=False,
                 outer_bc="dirichlet"):
        """filter_kind (with filter_params): 1 angular exponential filter of every
        component, (eta_c, alpha, order); 2 tensor-coupled ExpCheb filter,
        (eta_c, alpha, order); 3 tensor-coupled Heaviside filter, (eta_c,).
        interface_from_state: the characteristic projection and upwind choice
        at interfaces come from the state whose d_t u is being computed instead
        of the background u_bg.
        outer_bc: "dirichlet" (d_t u = 0 at the outer boundary) or
        "constraint_preserving" (gh.outer_constraint_preserving, with the
        normal and speeds from the state)."""
        self.shells = list(shells)
        self.grids = [_grid.ShellGrid(s.n_r, s.L, s.r_in, s.r_out) for s in self.shells]
        self.spheres = {}
        for s in self.shells:
            if s.L not in self.spheres:
                self.spheres[s.L] = _spec.Sphere(s.L)
        self.n_inst = 1 + max(s.instance for s in self.shells)
        self.npts = [g.npts for g in self.grids]
        self.offsets = np.concatenate([[0], np.cumsum(self.npts)])
        self.P = int(self.offsets[-1])
        self.filter_params = filter_params
        self.filter_kind = filter_kind if filter_params is not None else 0
        self.interface_from_state = bool(interface_from_state)
        if outer_bc not in ("dirichlet", "constraint_preserving"):
            raise ValueError("outer_bc must be 'dirichlet' or 'constraint_preserving'")
        self.outer_bc = outer_bc
        # interfaces: consecutive shells of one instance
        self.interfaces = []
        for k in range(len(self.shells) - 1):
            a, b = self.shells[k], self.shells[k + 1]
            if a.instance == b.instance:
                if a.L != b.L or abs(a.r_out - b.r_in) > 0.0:
                    raise ValueError("adjacent shells must share L and the interface radius")
                self.interfaces.append((k, k + 1))
        self.outer = [k for k in range(len(self.shells))
                      if k == len(self.shells) - 1 or self.shells[k + 1].instance != self.shells[k].instance]
        self.inner = [k for k in range(len(self.shells))
                      if k == 0 or self.shells[k - 1].instance != self.shells[k].instance]

    # -- layout helpers ------------------------------------------------------
    def split(self, v, ncomp):
        """Global array [ncomp * P] -> list of per-shell [ncomp, N_r, N_th, N_ph]."""
        out = []
        for k, g in enumerate(self.grids):
            o = ncomp * self.offsets[k]
            out.append(v[o:o + ncomp * g.npts].reshape(ncomp, g.n_r, g.n_th, g.n_ph))
        return out

    def join(self, blocks):
        return np.concatenate([b.ravel() for b in blocks])

    def xyz(self):
        """Collocation coordinates in layout order, shape [3, P]."""
        return np.concatenate([g.xyz() for g in self.grids], axis=1)

    def to_layout(self, a):
        """[ncomp, P] (points in shell order) -> flat layout [ncomp*P] (per-shell blocks)."""
        return np.concatenate([a[:, self.offsets[k]:self.offsets[k + 1]].ravel()
                               for k in range(len(self.grids))])

    def from_layout(self, v, ncomp):
        """Flat layout [ncomp*P] -> [ncomp, P]."""
        return np.concatenate([b.reshape(ncomp, -1) for b in self.split(v, ncomp)], axis=1)

    def per_point(self, blocks):
        """List of per-shell [ncomp, N_r, N_th, N_ph] -> [ncomp, P]."""
        return np.concatenate([b.reshape(b.shape[0], -1) for b in blocks], axis=1)

    # -- derivatives (the paper's DiffJac after the shell differentiator) ----
    def cartesian_derivs(self, k, ublk):
        """d_x, d_y, d_z of every component of one shell block [nc, N_r, N_th, N_ph].

        Radial and angular derivatives by transforms, then the Jacobian of the
        map (r, theta, phi) -> (x, y, z) (the paper's eq. DiffJac):
          d_x = s_th c_ph d_r + c_th c_ph / r d_th - s_ph / (r s_th) d_ph
          d_y = s_th s_ph d_r + c_th s_ph / r d_th + c_ph / (r s_th) d_ph
          d_z = c_th d_r - s_th / r d_th
        """
        g = self.grids[k]
        sph = self.spheres[g.L]
        dr = np.moveaxis(_spec.d_dxi(np.moveaxis(ublk, 1, 0)), 0, 1) * (2.0 / (g.r_out - g.r_in))
        dth = sph.d_dtheta(ublk)
        dph = sph.d_dphi(ublk)
        st, ct = np.sin(g.TH), np.cos(g.TH)
        sp, cp = np.sin(g.PH), np.cos(g.PH)
        r = g.R
        dx = st * cp * dr + ct * cp / r * dth - sp / (r * st) * dph
        dy = st * sp * dr + ct * sp / r * dth + cp / (r * st) * dph
        dz = ct * dr - st / r * dth
        return np.stack([dx, dy, dz])

    # -- right-hand side ----------------------------------------------------
    def rhs(self, u, H, dH, u_bg, gammas, apply_bc=True):
        """d_t u for the whole domain (interior algebra, then boundaries).

        u [50*P]; H [4*P]; dH [16*P]; u_bg [50*P]; gammas [n_inst, 3].
        """
        ub = self.split(u, 50)
        Hb = self.split(H, 4)
        dHb = self.split(dH, 16)
        out = []
        outer_du = {}
        for k, g in enumerate(self.grids):
            inst = self.shells[k].instance
            g0, g1, g2 = gammas[inst]
            du = self.cartesian_derivs(k, ub[k])
            dHk = dHb[k].reshape((4, 4) + dHb[k].shape[1:])
            out.append(_gh.rhs_pointwise(ub[k], du, Hb[k], dHk, g0, g1, g2))
            if k in self.outer:
                outer_du[k] = du[:, :, -1]
        if apply_bc:
            self.apply_bc(out, ub if self.interface_from_state else self.split(u_bg, 50), gammas,
                          state=ub, outer_du=outer_du)
        return self.join(out)

    def interface_projection(self, k, ubg_blk):
        """Unit normal s = +r_hat (g-normalised) at the outer face of shell k,
        with the metric of the given block (the background, or the state)."""
        g = self.grids[k]
        psi, _, _ = _gh.unpack_fields(ubg_blk[:, -1])
        geo = _gh.Geometry(psi)
        nhat = np.stack([np.sin(g.TH[-1]) * np.cos(g.PH[-1]),
                         np.sin(g.TH[-1]) * np.sin(g.PH[-1]),
                         np.cos(g.TH[-1])])
        s_lo, s_up = _gh.unit_normal(geo, nhat)
        return geo, s_lo, s_up

    def outer_projection(self, k, u_blk):
        """Unit normal s = +r_hat (normalised with the metric of u_blk) at the
        outer face of shell k."""
        return self.interface_projection(k, u_blk)

    def apply_bc(self, rhs_blocks, ubg_blocks, gammas, state=None, outer_du=None):
        """Boundary treatment of the per-shell d_t u blocks, in place.

        Paper (section on benchmarks of the overall code, closing remarks):
        internal boundaries exchange characteristic fields, the outer boundary
        gets a boundary condition, excision boundaries need none.  Readings:
        * interface (shell A inside, B outside, s = +r_hat normalised with the
          metric of ubg_blocks at A's outer face: the background u_bg, or the
          state itself when interface_from_state): project both sides' d_t u onto u^psi,
          u^0, u^+, u^-; take each of u^0, u^+-  from the upwind side (speed > 0:
          A, < 0: B, = 0: the average) and u^psi as the average of both sides;
          reconstruct and store the same d_t u on both sides;
        * outer boundary: Dirichlet, d_t u = 0 for all 50 fields, or (outer_bc
          "constraint_preserving") gh.outer_constraint_preserving with the
          normal and speeds from the state's metric at the face; that needs the
          state blocks and the Cartesian derivatives at the outer faces
          (state, outer_du[k] [3, 50, N_th, N_ph]);
        * inner (excision) boundary: nothing.
        """
        for (ka, kb) in self.interfaces:
            inst = self.shells[ka].instance
            g1, g2 = gammas[inst][1], gammas[inst][2]
            geo, s_lo, s_up = self.interface_projection(ka, ubg_blocks[ka])
            _, v0, vp, vm = _gh.char_speeds(geo, s_lo, g1)
            A = rhs_blocks[ka][:, -1]
            B = rhs_blocks[kb][:, 0]
            pa, u0a, upa, uma = _gh.char_fields(A, s_lo, s_up, g2)
            pb, u0b, upb, umb = _gh.char_fields(B, s_lo, s_up, g2)

            def pick(speed, xa, xb):
                wa = np.where(speed > 0, 1.0, np.where(speed < 0, 0.0, 0.5))
                return wa * xa + (1.0 - wa) * xb

            upsi = 0.5 * (pa + pb)
            u0 = pick(v0, u0a, u0b)
            up = pick(vp, upa, upb)
            um = pick(vm, uma, umb)
            new = _gh.char_reconstruct(upsi, u0, up, um, s_lo, g2)
            rhs_blocks[ka][:, -1] = new
            rhs_blocks[kb][:, 0] = new
        for k in self.outer:
            if self.outer_bc == "dirichlet":
                rhs_blocks[k][:, -1] = 0.0
                continue
            if state is None or outer_du is None or k not in outer_du:
                raise ValueError("the constraint-preserving outer treatment needs the state and its derivatives")
            inst = self.shells[k].instance
            g1, g2 = gammas[inst][1], gammas[inst][2]
            geo, s_lo, s_up = self.outer_projection(k, state[k])
            rhs_blocks[k][:, -1] = _gh.outer_constraint_preserving(
                rhs_blocks[k][:, -1], state[k][:, -1], outer_du[k], s_lo, s_up, geo, g1, g2)

    def excision_speeds(self, u_bg):
        """Speeds (u^0, u^+, u^-) at every inner boundary, normal s = -r_hat."""
        ubg = self.split(u_bg, 50)
        out = []
        for k in self.inner:
            g = self.grids[k]
            psi, _, _ = _gh.unpack_fields(ubg[k][:, 0])
            geo = _gh.Geometry(psi)
            nhat = -np.stack([np.sin(g.TH[0]) * np.cos(g.PH[0]),
                              np.sin(g.TH[0]) * np.sin(g.PH[0]), np.cos(g.TH[0])])
            s_lo, _ = _gh.unit_normal(geo, nhat)
            _, v0, vp, vm = _gh.char_speeds(geo, s_lo, 0.0)
            out.append(np.stack([v0, vp, vm]))
        return out

    # -- filter -------------------------------------------------------------
    def apply_filter(self, u):
        """The domain's angular filter on every shell: the exponential filter of
        every component (kind 1) or the tensor-coupled filter (kinds 2, 3)."""
        if self.filter_params is None:
            return u
        blocks = self.split(u, 50)
        out = []
        for k, g in enumerate(self.grids):
            if self.filter_kind == 1:
                eta_c, alpha, order = self.filter_params
                sig = _spec.exp_filter_sigma(g.L, eta_c, alpha, order)
                out.append(self.spheres[g.L].filter(blocks[k], sig))
            else:
                kind = "expcheb" if self.filter_kind == 2 else "heaviside"
                key = _tf.sigma_function(kind, g.L, self.filter_params)
                out.append(_tf.apply(self.spheres[g.L], blocks[k], key))
        return self.join(out)

    # -- time step ------------------------------------------------------------
    def dt_per_point(self, dt):
        """Per-instance time step broadcast to [50*P] in layout order."""
        return self.join([np.full((50, g.npts), dt[self.shells[k].instance])
                          for k, g in enumerate(self.grids)])

    def rk3_step(self, u, H, dH, u_bg, gammas, dt, rhs_fn=None):
        """One SSP-RK3 (Shu-Osher) step, then the angular filter if enabled.

        u1 = u + dt L(u); u2 = 3/4 u + 1/4 (u1 + dt L(u1));
        u_new = 1/3 u + 2/3 (u2 + dt L(u2)).
        """
        L = rhs_fn or (lambda v: self.rhs(v, H, dH, u_bg, gammas))
        h = self.dt_per_point(dt)
        u1 = u + h * L(u)
        u2 = 0.75 * u + 0.25 * (u1 + h * L(u1))
        un = (1.0 / 3.0) * u + (2.0 / 3.0) * (u2 + h * L(u2))
        return self.apply_filter(un)

    def instance_of_value(self):
        """Instance index of every value of a [50*P] field, layout order."""
        return self.join([np.full((50, g.npts), self.shells[k].instance)
                          for k, g in enumerate(self.grids)])

    def dp5_attempt(self, u, H, dH, u_bg, gammas, dt, atol, rtol, prev_rejected, rhs_fn=None):
        """One Dormand-Prince 5(4) attempt per instance with its own step dt[i].

        Every instance takes the seven stages with its dt; its error norm
        decides whether its fifth-order solution (filtered, if the filter is
        enabled) replaces its values, and sets its next dt (oracle/dp5.py).
        Returns (u_next, accepted[n_inst], dt_next[n_inst], err[n_inst]).
        """
        L = rhs_fn or (lambda v: self.rhs(v, H, dH, u_bg, gammas))
        h = self.dt_per_point(dt)
        u5, k = _dp5.stages(u, h, L)
        ev = _dp5.error_vector(k, h)
        owner = self.instance_of_value()
        acc = np.zeros(self.n_inst, dtype=bool)
        dt_next = np.array(dt, dtype=float).copy()
        errs = np.zeros(self.n_inst)
        for i in range(self.n_inst):
            m = owner == i
            errs[i] = _dp5.error_norm(ev[m], u[m], u5[m], atol, rtol)
            acc[i], scale = _dp5.control(errs[i], bool(prev_rejected[i]))
            dt_next[i] = dt[i] * scale
        new = self.apply_filter(u5)
        u_next = np.where(acc[owner], new, u)
        return u_next, acc, dt_next, errs

    # -- constraints ------------------------------------------------------------
    def constraints(self, u, H):
        """The 64 constraint components at every point, layout [64*P] per shell block."""
        ub = self.split(u, 50)
        Hb = self.split(H, 4)
        out = []
        for k in range(len(self.grids)):
            du = self.cartesian_derivs(k, ub[k])
            out.append(_gh.constraints_pointwise(ub[k], du, Hb[k]))
        return self.join(out)

    def constraint_norm(self, u, H):
        """Per instance ||C|| = sqrt(sum_p w_p sum_c C_c(p)^2 / sum_p w_p)."""
        Cb = self.split(self.constraints(u, H), 64)
        num = [0.0] * self.n_inst
        den = [0.0] * self.n_inst
        for k, g in enumerate(self.grids):
            w = g.volume_weights().reshape(g.n_r, g.n_th, g.n_ph)
            inst = self.shells[k].instance
            num[inst] = num[inst] + np.sum(w[None] * Cb[k] * Cb[k])
            den[inst] = den[inst] + np.sum(w)
        return np.array([np.sqrt(num[i] / den[i]) for i in range(self.n_inst)])
