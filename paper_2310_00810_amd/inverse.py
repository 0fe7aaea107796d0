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


__all__ = ["Adam", "History", "recover_constant_head", "recover_profile_and_tau", "darcy_permeability",
           "superficial_velocity", "pressure_gradient", "viscosity", "tau_from_viscosity", "reynolds",
           "math"]
