"""The evolution workloads: domains, damping parameters, time steps, initial data.

Each workload is an isolated Kerr-Schild black hole (or a batch of them) on a
stack of spherical shells, as in the paper's test problem (port overview: a
Kerr-Schild hole of mass m and spin chi on nested shells), at the sizes the
benchmarks use:

  single_shell       1 shell r in [1.8, 5], N_r = 11, L = 7 (8 x 16), Schwarzschild
                     M = 1, gamma = (1, -1, 1), dt = 0.01, no filter
  pulse_8shell       8 shells r in [1.8, 100] (geometric radii), N_r = 21,
                     L = 15 (16 x 32), Schwarzschild M = 1 plus a Gaussian
                     pulse in Pi_ab (amplitude 1e-3, width 2 at r = 10, seeded
                     random symmetric polarisation), angular exponential filter
                     on the top third of the degrees
  batched_64         64 Kerr holes, M ~ U[0.5, 2], chi ~ U[0, 0.9] along a
                     random axis, 4-12 shells each, N_r in {11,15,21,31} per
                     shell, L in {7,11,15,23} per hole (seeded)
  large_20shell      Kerr chi = 0.9, M = 1, 20 shells r in [1.4, 400], N_r = 33,
                     L = 31 (32 x 64), smooth random perturbation 1e-6
  large_20shell_batch  4 instances of the large domain (perturbation seeds 5..8),
                     the batch its adjoint is measured on

Time steps use the Courant factor of the single-shell case,
dt = 0.128 * (smallest radial spacing of the instance).
"""

import math

import numpy as np

from . import inputs

COURANT = 0.128
GAMMA_DEFAULT = (1.0, -1.0, 1.0)
FILTER_DEFAULT = (2.0 / 3.0, 36.0, 8.0)


def geometric_radii(r_in, r_out, n):
    rs = [r_in * (r_out / r_in) ** (i / n) for i in range(n + 1)]
    rs[0], rs[-1] = r_in, r_out
    return rs


def min_radial_spacing(n_r, r_in, r_out):
    return 0.5 * (r_out - r_in) * (1.0 - math.cos(math.pi / (n_r - 1)))


class Workload:
    """shells: list of (instance, n_r, L, r_in, r_out); holes: per instance (M, chi, axis)."""

    def __init__(self, name, shells, holes, gamma, dt, filter_params, n_steps, perturb):
        self.name = name
        self.shells = shells
        self.holes = holes
        self.n_inst = len(holes)
        self.gamma = np.array(gamma, dtype=float).reshape(self.n_inst, 3)
        self.dt = np.array(dt, dtype=float).reshape(self.n_inst)
        self.filter_params = filter_params
        self.n_steps = n_steps
        self.perturb = perturb

    @property
    def npoints(self):
        return sum(s[1] * 2 * (s[2] + 1) ** 2 for s in self.shells)

    def shells_of(self, inst):
        return [s for s in self.shells if s[0] == inst]

    def initial_data(self, xyz, offsets, device="cpu"):
        """Background fields, gauge source and perturbed initial state.

        xyz [3, P] collocation coordinates (layout point order) and the shell
        point offsets.  Returns numpy arrays in the flat layout:
        u0 [50 P], u_bg [50 P], H [4 P], dH [16 P].
        """
        P = xyz.shape[1]
        u_pts = np.zeros((50, P))
        H_pts = np.zeros((4, P))
        dH_pts = np.zeros((16, P))
        du_pts = np.zeros((50, P))
        for inst, (M, chi, axis) in enumerate(self.holes):
            ks = [k for k, s in enumerate(self.shells) if s[0] == inst]
            lo, hi = offsets[ks[0]], offsets[ks[-1] + 1]
            ex = inputs.kerr_schild(xyz[:, lo:hi], M=M, chi=chi, axis=axis, device=device)
            u_pts[:, lo:hi] = ex["u"]
            H_pts[:, lo:hi] = ex["H"]
            dH_pts[:, lo:hi] = ex["dH"]
            if self.perturb is not None:
                du_pts[:, lo:hi] = self.perturb(xyz[:, lo:hi], inst)
        to = lambda a: to_layout(a, self.shells, offsets)
        return to(u_pts + du_pts), to(u_pts), to(H_pts), to(dH_pts)


def to_layout(a, shells, offsets):
    """[ncomp, P] (points in shell order) -> flat [ncomp * P] shell-blocked layout."""
    return np.concatenate([a[:, offsets[k]:offsets[k + 1]].ravel() for k in range(len(shells))])


def from_layout(v, ncomp, shells, offsets):
    blocks = []
    for k in range(len(shells)):
        n = offsets[k + 1] - offsets[k]
        blocks.append(v[ncomp * offsets[k]: ncomp * offsets[k + 1]].reshape(ncomp, n))
    return np.concatenate(blocks, axis=1)


def single_shell():
    shells = [(0, 11, 7, 1.8, 5.0)]
    return Workload("single_shell", shells, [(1.0, 0.0, (0.0, 0.0, 1.0))], [GAMMA_DEFAULT],
                    [0.01], None, 10, None)


def pulse_8shell(seed=0, n_steps=1000):
    rs = geometric_radii(1.8, 100.0, 8)
    shells = [(0, 21, 15, rs[i], rs[i + 1]) for i in range(8)]
    dt = COURANT * min(min_radial_spacing(s[1], s[3], s[4]) for s in shells)
    pert = lambda xyz, inst: inputs.gaussian_pulse_Pi(xyz, 1e-3, 10.0, 2.0, seed)
    return Workload("pulse_8shell", shells, [(1.0, 0.0, (0.0, 0.0, 1.0))], [GAMMA_DEFAULT], [dt],
                    FILTER_DEFAULT, n_steps, pert)


def batched_64(seed=3, n_inst=64):
    rng = np.random.default_rng(seed)
    shells, holes, dts = [], [], []
    for inst in range(n_inst):
        M = rng.uniform(0.5, 2.0)
        chi = rng.uniform(0.0, 0.9)
        axis = rng.standard_normal(3)
        axis = tuple(axis / np.linalg.norm(axis))
        ns = int(rng.integers(4, 13))
        L = int(rng.choice([7, 11, 15, 23]))
        r_in = 0.9 * M * (1.0 + math.sqrt(1.0 - chi * chi))
        rs = geometric_radii(r_in, 50.0 * M, ns)
        sh = [(inst, int(rng.choice([11, 15, 21, 31])), L, rs[i], rs[i + 1]) for i in range(ns)]
        shells += sh
        holes.append((M, chi, axis))
        dts.append(COURANT * min(min_radial_spacing(s[1], s[3], s[4]) for s in sh))
    return Workload("batched_64", shells, holes, [GAMMA_DEFAULT] * n_inst, dts, None, 1000, None)


def large_20shell(seed=5):
    rs = geometric_radii(1.4, 400.0, 20)
    shells = [(0, 33, 31, rs[i], rs[i + 1]) for i in range(20)]
    dt = COURANT * min(min_radial_spacing(s[1], s[3], s[4]) for s in shells)
    pert = lambda xyz, inst: inputs.smooth_random_field(xyz, 1e-6, seed, 10, 8.0)
    return Workload("large_20shell", shells, [(1.0, 0.9, (0.0, 0.0, 1.0))], [GAMMA_DEFAULT], [dt],
                    None, 2000, pert)


def large_20shell_batch(n_inst=4, seed=5):
    """n_inst copies of the large domain, instance i perturbed with seed + i."""
    one = large_20shell(seed)
    shells = [(i,) + tuple(sh[1:]) for i in range(n_inst) for sh in one.shells]
    pert = lambda xyz, inst: inputs.smooth_random_field(xyz, 1e-6, seed + inst, 10, 8.0)
    return Workload("large_20shell_batch", shells, [one.holes[0]] * n_inst, [GAMMA_DEFAULT] * n_inst,
                    [one.dt[0]] * n_inst, None, one.n_steps, pert)


WORKLOADS = {"single_shell": single_shell, "pulse_8shell": pulse_8shell,
             "batched_64": batched_64, "large_20shell": large_20shell,
             "large_20shell_batch": large_20shell_batch}
