"""Host-side inverse-problem drivers on top of the GPU solver.

The workflow of Section 2.2 (initialise, run T steps, evaluate the loss,
back-propagate, update the parameter with a gradient-based optimiser) and
the permeability estimate of Section 3.2 (Darcy's law, Eq. 12, fitted along
the sequence of forward solutions the optimiser visits).

Parameters are density deviations drho = rho - 1 and the relaxation time
tau.  Updates descend the loss (p <- p - lr * dL/dp).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch


@dataclass
class Adam:
    """Adam on a flat float64 parameter vector."""
    lr: float
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-12
    m: np.ndarray | None = None
    v: np.ndarray | None = None
    t: int = 0

    def step(self, p, g):
        if self.m is None:
            self.m = np.zeros_like(p)
            self.v = np.zeros_like(p)
        self.t += 1
        self.m = self.beta1 * self.m + (1 - self.beta1) * g
        self.v = self.beta2 * self.v + (1 - self.beta2) * g * g
        mh = self.m / (1 - self.beta1 ** self.t)
        vh = self.v / (1 - self.beta2 ** self.t)
        return p - self.lr * mh / (np.sqrt(vh) + self.eps)


@dataclass
class History:
    loss: list = field(default_factory=list)
    params: list = field(default_factory=list)
    grads: list = field(default_factory=list)
    flux: list = field(default_factory=list)


def recover_constant_head(solver, tau, drho0, drho_out=0.0, max_iter=30, rtol=None, true_drho=None,
                          armijo_c=1e-4, step0=None):
    """Gradient descent with Armijo backtracking on a scalar inlet density
    deviation (one instance).  The first trial step is the Newton-like step
    of a quadratic model through the current point (L / L'), halved until the
    Armijo condition holds.  Stops when |drho - true| <= rtol * |true| (if a
    truth is given) or after max_iter iterations."""
    h = History()
    p = float(drho0)
    L = solver.forward(tau, p, drho_out, record_tape=True)[0]
    for it in range(max_iter):
        solver.adjoint()
        g = solver.grad()["drho_in"][0]
        h.loss.append(L)
        h.params.append(p)
        h.grads.append(g)
        _, u = solver.macro()
        h.flux.append(float(u[:, 0].double().sum().item()))
        if true_drho is not None and rtol is not None and abs(p - true_drho) <= rtol * abs(true_drho):
            break
        if g == 0.0:
            break
        step = 2.0 * L / g if step0 is None else step0 * np.sign(g)
        for _ in range(40):
            pn = p - step
            Ln = solver.forward(tau, pn, drho_out, record_tape=True)[0]
            if Ln <= L - armijo_c * abs(step * g):
                break
            step *= 0.5
        p, L = pn, Ln
    return p, h


def recover_profile_and_tau(solver, tau0, drho_in0, drho_out=0.0, iters=20, lr_in=2e-4, lr_tau=2e-2):
    """Joint Adam recovery of a per-node inlet profile and tau (one
    instance): returns (profile, tau, history)."""
    h = History()
    p = np.asarray(drho_in0, np.float64).copy()
    tau = float(tau0)
    opt_in, opt_tau = Adam(lr_in), Adam(lr_tau)
    for it in range(iters):
        L = solver.forward(tau, p, drho_out, record_tape=True)[0]
        solver.adjoint()
        g = solver.grad()
        h.loss.append(L)
        h.params.append((p.copy(), tau))
        h.grads.append((g["drho_in"].copy(), g["dtau"][0]))
        p = opt_in.step(p, g["drho_in"])
        tau = float(opt_tau.step(np.array([tau]), g["dtau"])[0])
        tau = max(tau, 0.5 + 1e-3)
    return p, tau, h


def darcy_permeability(q_superficial, grad_p, rho_mean, nu):
    """Darcy's law (Eq. 12) k = rho nu q / |dp/dx|, fitted through the origin
    over several (q, dp/dx) pairs:  k = rho nu sum(q g) / sum(g g)."""
    q = np.asarray(q_superficial, np.float64)
    g = np.abs(np.asarray(grad_p, np.float64))
    slope = float(np.sum(q * g) / np.sum(g * g))
    return rho_mean * nu * slope


def darcy_fit(solver, tau, drhos, solid, tol=1e-6, max_steps=200_000):
    """Darcy permeability (Eq. 12) of one medium from its steady states at the
    inlet densities 1 + drhos (outlet 1): superficial velocity against the
    mean pressure gradient, fitted through the origin.  solver: a one-instance
    Solver of the medium; solid: its (nz, ny, nx) mask.  Returns (k, points)
    with points = [(drho, q, grad_p, rho_mean, steps)]."""
    nz, ny, nx = solid.shape
    fl = torch.from_numpy(solid.reshape(-1) == 0).to(solver.device)
    pts = []
    for d in drhos:
        solver.set_initial(None, None)
        steps, _ = solver.run_to_residual(tau, float(d), 0.0, tol=tol, max_steps=max_steps)
        drho, u = solver.macro(mean2=True)
        q = superficial_velocity(u[:, 0].double().cpu().numpy(), nx * ny * nz)
        rho = 1.0 + float(drho[fl].double().mean().item())
        pts.append((float(d), q, pressure_gradient(float(d), 0.0, nx), rho, steps))
    k = darcy_permeability([p[1] for p in pts], [p[2] for p in pts], float(np.mean([p[3] for p in pts])),
                           viscosity(tau))
    return k, pts


def superficial_velocity(u_x, n_nodes):
    """Mean of u_x over all nodes (solid nodes count as zero)."""
    return float(np.sum(u_x) / n_nodes)


def pressure_gradient(drho_in, drho_out, nx):
    """Mean pressure gradient cs^2 (rho_in - rho_out) / (nx - 1) with p = rho / 3."""
    return (drho_in - drho_out) / 3.0 / (nx - 1)


def viscosity(tau):
    """Lattice kinematic viscosity (Eq. 9): nu = (tau - 1/2) / 3."""
    return (tau - 0.5) / 3.0


def tau_from_viscosity(nu):
    return 3.0 * nu + 0.5


def reynolds(U, D, nu):
    """Eq. 11: Re = U D / (2 nu)."""
    return U * D / (2.0 * nu)


def carman_kozeny(porosity, d_p, phi_s=1.0, phi_ck=180.0):
    """Carman-Kozeny permeability (Eq. 8): k = phi_s^2 eps^3 D_p^2 / (Phi_CK (1 - eps)^2),
    with eps the porosity, D_p the mean grain diameter, phi_s the sphericity
    and Phi_CK the Kozeny factor (180 for a packing of spheres)."""
    e = float(porosity)
    return phi_s ** 2 * e ** 3 * d_p ** 2 / (phi_ck * (1.0 - e) ** 2)


def kozeny_factor(tortuosity, phi=90.0):
    """Kozeny factor from the tortuosity L_e / L of the streamlines (Section
    3.3): Phi_CK = Phi (L_e / L)^2, Phi = 90 for spherical grains."""
    return phi * tortuosity ** 2


def physical_permeability(k_lattice, dx):
    """Lattice permeability (lu^2) in m^2 for a lattice spacing dx (m per lu)."""
    return k_lattice * dx ** 2


def lattice_time_step(nu_lattice, dx, nu_physical=1e-6):
    """Seconds per time step that make the lattice viscosity the physical one:
    nu_phys = nu_lattice dx^2 / dt (water: 1e-6 m^2/s)."""
    return nu_lattice * dx ** 2 / nu_physical


def spline_basis(n_nodes, n_knots):
    """Matrix B (n_nodes x n_knots) of the natural cubic spline through
    n_knots equally spaced knots spanning the n_nodes inlet nodes: the
    profile is B @ knot_values, and a gradient with respect to the profile
    maps to the knots as B.T @ g (Section 3.2 draws the inlet pressure as a
    cubic spline).  Natural: zero second derivative at the end knots."""
    if n_knots < 2 or n_nodes < 1:
        raise ValueError("need at least two knots and one node")
    xk = np.linspace(0.0, n_nodes - 1.0, n_knots)
    h = np.diff(xk)
    n = n_knots
    # second derivatives M of the spline through unit knot vectors: A M = R v
    A = np.zeros((n, n))
    R = np.zeros((n, n))
    A[0, 0] = A[-1, -1] = 1.0
    for i in range(1, n - 1):
        A[i, i - 1], A[i, i], A[i, i + 1] = h[i - 1] / 6.0, (h[i - 1] + h[i]) / 3.0, h[i] / 6.0
        R[i, i - 1], R[i, i], R[i, i + 1] = 1.0 / h[i - 1], -1.0 / h[i - 1] - 1.0 / h[i], 1.0 / h[i]
    Mv = np.linalg.solve(A, R)                       # n x n: second derivatives per unit knot
    x = np.arange(n_nodes, dtype=np.float64)
    j = np.clip(np.searchsorted(xk, x, side="right") - 1, 0, n - 2)
    a = (xk[j + 1] - x) / h[j]
    b = (x - xk[j]) / h[j]
    B = np.zeros((n_nodes, n))
    rows = np.arange(n_nodes)
    B[rows, j] += a
    B[rows, j + 1] += b
    c2 = h[j] ** 2 / 6.0
    B += ((a ** 3 - a) * c2)[:, None] * Mv[j] + ((b ** 3 - b) * c2)[:, None] * Mv[j + 1]
    return B


__all__ = ["Adam", "History", "recover_constant_head", "recover_profile_and_tau", "darcy_permeability",
           "superficial_velocity", "pressure_gradient", "viscosity", "tau_from_viscosity", "reynolds",
           "carman_kozeny", "kozeny_factor", "physical_permeability", "lattice_time_step", "spline_basis",
           "math"]
