"""Python front end of the MI355X differentiable lattice Boltzmann library.

``Solver`` owns one workspace (a torch uint8 device tensor) and one handle of
liblbm.so; PyTorch supplies device memory and the stream, the library runs
every step of the method.  ``LBMLoss`` and ``LBMField`` expose the forward
map to torch.autograd with the library's hand-written adjoint as backward.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as C

_LOSS = {"vec": C.LOSS_VEC, "norm": C.LOSS_NORM}
_SCALE = {"sum": C.SCALE_SUM, "mean": C.SCALE_MEAN_FLUID}
_INLET = {"const": C.INLET_CONST, "profile": C.INLET_PROFILE}
_BC = {"pressure": C.BC_PRESSURE, "periodic": C.BC_PERIODIC, "wall": C.BC_WALL, "abb": C.BC_ABB,
       "velocity": C.BC_VELOCITY}
# D2Q9 multiple-relaxation-time rates of (rho, e, eps, jx, qx, jy, qy, pxx, pxy):
# conserved moments 1.0, the energy / flux rates of Lallemand & Luo; the two
# stress rates are 1/tau.
MRT_RATES = (1.0, 1.64, 1.54, 1.0, 1.9, 1.0, 1.9, 1.0, 1.0)


@dataclass
class Instance:
    """One lattice: shape (nx, ny, nz), optional solid mask (nz, ny, nx),
    loss weights (nz, ny, nx) and target velocity (nz, ny, nx, D), or one
    target per loss frame (frames, nz, ny, nx, D) for a time-windowed loss."""
    nx: int
    ny: int
    nz: int = 1
    solid: np.ndarray | None = None
    roi: np.ndarray | None = None
    target_u: np.ndarray | None = None

    @property
    def nodes(self):
        return self.nx * self.ny * self.nz


def _bc(v):
    return _BC[v] if isinstance(v, str) else int(v)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _tptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Solver:
    """A differentiable LBM problem on one GPU.

    lattice: 9 or 19.  instances: list of Instance (a batch of independent
    lattices).  bc: boundary kind per axis (x, y, z).  steps: T.
    ckpt_interval: K (0 = ceil(sqrt(T))).  tape: reserve the adjoint tape.
    collision: "bgk" or (D2Q9) "mrt" with mrt_rates.  resident_segments: the
    taped forward keeps the states of its last R segments (K-1 states each), so
    the reverse sweep recomputes only the others; "max" takes as many as fit in
    the free device memory less `reserve_bytes`.  loss_frames, loss_stride:
    time-windowed loss over the states after steps T - (frames - 1 - m)
    stride (the instances then carry one target per frame)."""

    def __init__(self, lattice, instances, bc=("pressure", "wall", "periodic"), steps=1,
                 ckpt_interval=0, tape=False, loss_kind="vec", loss_scale="sum",
                 inlet_mode="const", device="cuda", stream=None, collision="bgk", mrt_rates=MRT_RATES,
                 resident_segments=1, reserve_bytes=8 << 30, loss_frames=1, loss_stride=1):
        self.q = int(lattice)
        self.D = 2 if self.q == 9 else 3
        self.instances = list(instances)
        self.n_inst = len(self.instances)
        self.steps = int(steps)
        self.inlet_mode = inlet_mode
        self.device = torch.device(device)
        self._keep = []
        arr = (C.lbm_instance * self.n_inst)()
        for k, ins in enumerate(self.instances):
            arr[k].nx, arr[k].ny, arr[k].nz = ins.nx, ins.ny, ins.nz
            arr[k].solid = self._host(ins.solid, np.uint8, (ins.nz, ins.ny, ins.nx))
            arr[k].roi = self._host(ins.roi, np.float32, (ins.nz, ins.ny, ins.nx))
            arr[k].target_u = self._host(ins.target_u, np.float32,
                                         (max(int(loss_frames), 1), ins.nz, ins.ny, ins.nx, self.D))
        self._inst_arr = arr
        self.problem = C.lbm_problem(self.q, self.n_inst, arr, _bc(bc[0]), _bc(bc[1]), _bc(bc[2]),
                                     self.steps, int(ckpt_interval), int(bool(tape)), _LOSS[loss_kind],
                                     _SCALE[loss_scale], _INLET[inlet_mode],
                                     C.COLL_MRT if collision == "mrt" else C.COLL_BGK,
                                     (ctypes.c_double * 9)(*[float(r) for r in mrt_rates]), 1,
                                     int(loss_frames), int(loss_stride))
        L = C.lib()
        nbytes = ctypes.c_size_t(0)
        C.check(L.lbm_workspace_bytes(ctypes.byref(self.problem), ctypes.byref(nbytes)), "lbm_workspace_bytes")
        if resident_segments == "max":
            # one more resident segment costs the difference of two workspace sizes
            base_bytes = int(nbytes.value)
            self.problem.resident_segments = 2
            C.check(L.lbm_workspace_bytes(ctypes.byref(self.problem), ctypes.byref(nbytes)), "lbm_workspace_bytes")
            per_seg = int(nbytes.value) - base_bytes
            free = torch.cuda.mem_get_info(self.device)[0]
            r = 1 if per_seg <= 0 else 1 + max(0, (free - reserve_bytes - base_bytes) // per_seg)
            self.problem.resident_segments = int(max(1, r))
        else:
            self.problem.resident_segments = int(resident_segments)
        K = int(ckpt_interval) if int(ckpt_interval) > 0 else int(np.ceil(np.sqrt(self.steps)))
        n_seg = -(-self.steps // min(K, self.steps))
        self.problem.resident_segments = min(max(self.problem.resident_segments, 1), n_seg)
        C.check(L.lbm_workspace_bytes(ctypes.byref(self.problem), ctypes.byref(nbytes)), "lbm_workspace_bytes")
        self.resident_segments = self.problem.resident_segments
        self.workspace_bytes = int(nbytes.value)
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        C.check(L.lbm_init(ctypes.byref(h), ctypes.byref(self.problem), ctypes.c_void_p(self._ws_ptr),
                           self.workspace_bytes, ctypes.c_void_p(self.stream.cuda_stream)), "lbm_init")
        self.handle = h
        self._destroy = L.lbm_destroy  # bound now: module globals may be gone when __del__ runs at exit
        self._keep.clear()  # host arrays were copied by lbm_init

    def _host(self, a, dtype, shape):
        if a is None:
            return None
        a = np.ascontiguousarray(np.asarray(a, dtype=dtype).reshape(shape))
        self._keep.append(a)
        return a.ctypes.data_as(ctypes.c_void_p)

    def __del__(self):
        h, destroy = getattr(self, "handle", None), getattr(self, "_destroy", None)
        if h is not None and destroy is not None:
            destroy(h)
            self.handle = None

    # ------------------------------------------------------------ params --
    @property
    def nodes(self):
        return sum(i.nodes for i in self.instances)

    @property
    def face_nodes(self):
        return [i.ny * i.nz for i in self.instances]

    def _params(self, tau, drho_in, drho_out):
        tau = np.ascontiguousarray(np.broadcast_to(np.asarray(tau, np.float64), (self.n_inst,)))
        if self.inlet_mode == "profile":
            din = np.ascontiguousarray(np.asarray(drho_in, np.float64).reshape(-1))
            if din.size != sum(self.face_nodes):
                raise ValueError("profile inlet needs one value per inlet node")
        else:
            din = np.ascontiguousarray(np.broadcast_to(np.asarray(drho_in, np.float64), (self.n_inst,)))
        dout = np.ascontiguousarray(np.broadcast_to(np.asarray(drho_out, np.float64), (self.n_inst,)))
        self._prm_keep = (tau, din, dout)
        return C.lbm_params(_dptr(tau), _dptr(din), _dptr(dout))

    # ---------------------------------------------------------- calls --
    def _order(self, *tensors):
        """Orders the library's stream after torch's current stream (where the
        caller's tensors were produced or allocated) and marks the tensors as
        used on the library's stream, so that neither a pending producer nor
        the caching allocator races with the library's kernels."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)
            for t in tensors:
                if t is not None:
                    t.record_stream(self.stream)

    def forward(self, tau, drho_in, drho_out, record_tape=False, want_loss=True):
        """Runs T steps from the initial state; returns the per-instance
        losses (numpy float64) or None."""
        prm = self._params(tau, drho_in, drho_out)
        out = np.zeros(self.n_inst) if want_loss else None
        C.check(C.lib().lbm_forward(self.handle, ctypes.byref(prm), int(bool(record_tape)),
                                    _dptr(out) if want_loss else None), "lbm_forward")
        return out

    def adjoint(self, seed_du=None):
        if seed_du is not None:
            seed_du = seed_du.to(device=self.device, dtype=torch.float32).contiguous()
            self._order(seed_du)
        C.check(C.lib().lbm_adjoint(self.handle, _tptr(seed_du)), "lbm_adjoint")

    def grad(self):
        n_in = sum(self.face_nodes) if self.inlet_mode == "profile" else self.n_inst
        din = np.zeros(n_in)
        dtau = np.zeros(self.n_inst)
        dout = np.zeros(self.n_inst)
        C.check(C.lib().lbm_grad(self.handle, _dptr(din), _dptr(dtau), _dptr(dout)), "lbm_grad")
        return dict(drho_in=din, dtau=dtau, drho_out=dout)

    def set_initial(self, drho=None, u=None):
        drho = drho.to(self.device, torch.float32).contiguous() if drho is not None else None
        u = u.to(self.device, torch.float32).contiguous() if u is not None else None
        self._order(drho, u)
        C.check(C.lib().lbm_set_initial(self.handle, _tptr(drho), _tptr(u)), "lbm_set_initial")

    def set_populations(self, fbar):
        fbar = fbar.to(self.device, torch.float32).contiguous()
        self._order(fbar)
        C.check(C.lib().lbm_set_populations(self.handle, _tptr(fbar)), "lbm_set_populations")

    def get_populations(self, which="state"):
        out = torch.empty(self.q * self.nodes, dtype=torch.float32, device=self.device)
        self._order(out)
        k = C.POP_STATE if which == "state" else C.POP_ADJOINT
        C.check(C.lib().lbm_get_populations(self.handle, k, _tptr(out)), "lbm_get_populations")
        self.stream.synchronize()
        return out

    def macro(self, mean2=False):
        drho = torch.empty(self.nodes, dtype=torch.float32, device=self.device)
        u = torch.empty(self.nodes * self.D, dtype=torch.float32, device=self.device)
        self._order(drho, u)
        C.check(C.lib().lbm_get_macro(self.handle, _tptr(drho), _tptr(u), int(bool(mean2))), "lbm_get_macro")
        self.stream.synchronize()
        return drho, u.view(self.nodes, self.D)

    def run_to_residual(self, tau, drho_in, drho_out, tol=1e-6, max_steps=100_000, check_every=100):
        prm = self._params(tau, drho_in, drho_out)
        steps = ctypes.c_int(0)
        r = ctypes.c_double(0.0)
        C.check(C.lib().lbm_run_to_residual(self.handle, ctypes.byref(prm), float(tol), int(max_steps),
                                            int(check_every), ctypes.byref(steps), ctypes.byref(r)),
                "lbm_run_to_residual")
        return steps.value, r.value

    def residuals(self):
        """Per-instance residuals of the last run_to_residual check (numpy)."""
        out = np.zeros(self.n_inst)
        C.check(C.lib().lbm_get_residuals(self.handle, _dptr(out)), "lbm_get_residuals")
        return out

    def checkpoint(self, c):
        """Checkpoint c (the state after c K steps of the taped forward,
        c = 1 .. n_seg - 1) as a float32 view into the workspace."""
        ptr, nbytes = ctypes.c_void_p(), ctypes.c_size_t(0)
        C.check(C.lib().lbm_checkpoint(self.handle, int(c), ctypes.byref(ptr), ctypes.byref(nbytes)),
                "lbm_checkpoint")
        off = ptr.value - self.workspace.data_ptr()
        return self.workspace[off:off + nbytes.value].view(torch.float32)

    def set_graphs(self, enable=True):
        C.check(C.lib().lbm_set_graphs(self.handle, int(enable)), "lbm_set_graphs")

    def set_timing(self, enable=True, reset=True):
        C.check(C.lib().lbm_set_timing(self.handle, int(enable), int(reset)), "lbm_set_timing")

    def timing(self):
        t = C.lbm_timing()
        C.check(C.lib().lbm_get_timing(self.handle, ctypes.byref(t)), "lbm_get_timing")
        return {k: getattr(t, k) for k, _ in t._fields_}

    def split(self, flat):
        """Splits a per-node concatenated array into per-instance views."""
        out, o = [], 0
        for ins in self.instances:
            out.append(flat[o:o + ins.nodes])
            o += ins.nodes
        return out


class LBMLoss(torch.autograd.Function):
    """loss = LBMLoss.apply(solver, drho_in, tau, drho_out)

    drho_in: (n_inst,) or (sum of inlet nodes,) float64 CPU tensor; tau and
    drho_out: (n_inst,).  Forward: taped lbm_forward; backward: lbm_adjoint +
    lbm_grad with the built-in loss."""

    @staticmethod
    def forward(ctx, solver, drho_in, tau, drho_out):
        ctx.solver = solver
        loss = solver.forward(tau.detach().cpu().numpy(), drho_in.detach().cpu().numpy(),
                              drho_out.detach().cpu().numpy(), record_tape=True)
        return torch.as_tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gout):
        s = ctx.solver
        s.adjoint(None)
        g = s.grad()
        go = gout.detach().cpu().numpy()
        if s.inlet_mode == "profile":
            scale_in = np.repeat(go, s.face_nodes)
        else:
            scale_in = go
        return (None, torch.as_tensor(g["drho_in"] * scale_in), torch.as_tensor(g["dtau"] * go),
                torch.as_tensor(g["drho_out"] * go))


class LBMField(torch.autograd.Function):
    """u = LBMField.apply(solver, drho_in, tau, drho_out): the final velocity
    u(T) as a (nodes, D) device tensor; backward seeds the adjoint with
    dL/du(T) from any torch loss."""

    @staticmethod
    def forward(ctx, solver, drho_in, tau, drho_out):
        ctx.solver = solver
        solver.forward(tau.detach().cpu().numpy(), drho_in.detach().cpu().numpy(),
                       drho_out.detach().cpu().numpy(), record_tape=True, want_loss=False)
        _, u = solver.macro(mean2=False)
        return u.clone()

    @staticmethod
    def backward(ctx, gu):
        s = ctx.solver
        s.adjoint(gu.contiguous())
        g = s.grad()
        return (None, torch.as_tensor(g["drho_in"]), torch.as_tensor(g["dtau"]),
                torch.as_tensor(g["drho_out"]))
