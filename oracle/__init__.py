"""FP64 CPU oracle of the differentiable lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY: this package may be imported by ``tests/``, by the
package's ``smoke()`` check and by the CPU-baseline leg of ``bench.py``; the
product path never calls it.  It shares no code with the GPU path.

The arithmetic lives in plain C (``lbm_oracle.c``, ``conv_oracle.c``); this
module only marshals numpy arrays.

Array conventions (all float64, C order):
  populations f : (nz, ny, nx, Q)      -- array of structures, unshifted f_i
  rho           : (nz, ny, nx)
  u             : (nz, ny, nx, 3)      -- u_z = 0 in 2D
  face densities: (nz, ny)             -- one absolute density per face node
  solid         : (nz, ny, nx) uint8   -- nonzero = solid

Velocity ordering
  D2Q9 : (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)
  D3Q19: rest, +x -x +y -y +z -z, (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0),
         (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1), (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liblbm_oracle.so")

BC_PRESSURE, BC_PERIODIC, BC_WALL, BC_ABB, BC_VELOCITY = 0, 1, 2, 3, 4
# D2Q9 multiple-relaxation-time rates (rho, e, eps, jx, qx, jy, qy, pxx, pxy);
# the stress rates are replaced by 1/tau.  Conserved moments 1.0; the others
# from the commonly used set of Lallemand & Luo.
MRT_RATES = (1.0, 1.64, 1.54, 1.0, 1.9, 1.0, 1.9, 1.0, 1.0)
LOSS_VEC, LOSS_NORM = 0, 1

C2 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0],
               [1, 1, 0], [-1, 1, 0], [-1, -1, 0], [1, -1, 0]])
W2 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
C3 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
               [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
               [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
               [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
W3 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def velocities(q):
    """(c, w) of the lattice with q velocities."""
    return (C2, W2) if q == 9 else (C3, W3)


_lib = None


def load(path):
    """Use the oracle library at path (a build of the same sources, e.g. the
    -O3 -march=native copy of ``build.build(native=True)``) from now on."""
    global _lib
    _lib = ctypes.CDLL(path)
    return _lib


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            from . import build as _b
            _b.build()
        _lib = ctypes.CDLL(LIBPATH)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)


def _p(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Lattice:
    """Geometry of one lattice: q in {9, 19}, shape (nz, ny, nx), per-axis
    boundary kind (x, y, z), an optional solid mask and, for D2Q9, optional
    multiple-relaxation-time rates (None = BGK)."""

    def __init__(self, q, nx, ny, nz=1, bc=(BC_PRESSURE, BC_WALL, BC_PERIODIC), solid=None, mrt=None):
        self.q, self.nx, self.ny, self.nz = int(q), int(nx), int(ny), int(nz)
        self.bc = (ctypes.c_int * 3)(*bc)
        self.bc_tuple = tuple(bc)
        if solid is None:
            solid = np.zeros((nz, ny, nx), np.uint8)
        self.solid = np.ascontiguousarray(solid.reshape(nz, ny, nx), dtype=np.uint8)
        self.mrt = None if mrt is None else _f64(np.asarray(mrt, np.float64).reshape(9))

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def args(self):
        return (self.q, self.nx, self.ny, self.nz, self.bc,
                self.solid.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), _p(self.mrt))

    def face(self, value):
        """Broadcast a scalar or (nz, ny) array to a face density array."""
        return _f64(np.broadcast_to(np.asarray(value, np.float64), (self.nz, self.ny)))

    def fluid(self):
        return self.solid == 0


def equilibrium(q, rho, u):
    out = np.zeros(q)
    lib().orc_equilibrium(q, ctypes.c_double(rho), _p(_f64(u)), _p(out))
    return out


def init_eq(lat, rho, u):
    rho = _f64(np.broadcast_to(np.asarray(rho, np.float64), lat.shape))
    u = _f64(np.broadcast_to(np.asarray(u, np.float64), lat.shape + (3,)))
    f = np.zeros(lat.shape + (lat.q,))
    lib().orc_init_eq(*lat.args(), _p(rho), _p(u), _p(f))
    return f


def collide(lat, tau, f):
    f = _f64(f).copy()
    lib().orc_collide(*lat.args(), ctypes.c_double(tau), _p(f))
    return f


def stream(lat, f):
    f = _f64(f)
    g = np.zeros_like(f)
    lib().orc_stream(*lat.args(), _p(f), _p(g))
    return g


def zouhe(lat, rho_in, rho_out, g):
    g = _f64(g).copy()
    lib().orc_zouhe(*lat.args(), _p(lat.face(rho_in)), _p(lat.face(rho_out)), _p(g))
    return g


def abb(lat, rho_in, rho_out, fs, g):
    """Anti-bounce-back pass (Eq. 6) on the x faces: fills the unknown slots of
    the streamed state g from the post-collision state fs."""
    g = _f64(g).copy()
    lib().orc_abb(*lat.args(), _p(lat.face(rho_in)), _p(lat.face(rho_out)), _p(_f64(fs)), _p(g))
    return g


def abb_adj(lat, rho_in, rho_out, fs, gbar):
    """(gbar with the unknown slots cleared, the pass's contribution to
    dL/dfs, d/drho_in, d/drho_out) of the anti-bounce-back pass."""
    gbar = _f64(gbar).copy()
    fsbar = np.zeros(lat.shape + (lat.q,))
    din = np.zeros((lat.nz, lat.ny))
    dout = np.zeros((lat.nz, lat.ny))
    lib().orc_abb_adj(*lat.args(), _p(lat.face(rho_in)), _p(lat.face(rho_out)), _p(_f64(fs)),
                      _p(gbar), _p(fsbar), _p(din), _p(dout))
    return gbar, fsbar, din, dout


def run(lat, tau, rho_in, rho_out, f0, T):
    """T steps (collide, stream, boundary pass) from f0; returns the final state."""
    f = _f64(f0).copy()
    lib().orc_run(*lat.args(), ctypes.c_double(tau), _p(lat.face(rho_in)),
                  _p(lat.face(rho_out)), _p(f), ctypes.c_int(T))
    return f


def macro(lat, f):
    rho = np.zeros(lat.shape)
    u = np.zeros(lat.shape + (3,))
    lib().orc_macro(*lat.args(), _p(_f64(f)), _p(rho), _p(u))
    return rho, u


def loss(lat, f, target_u, weight=None, kind=LOSS_VEC, scale=1.0):
    fn = lib().orc_loss
    fn.restype = ctypes.c_double
    w = _f64(weight) if weight is not None else None
    return fn(*lat.args(), _p(_f64(f)), _p(_f64(target_u)), _p(w), ctypes.c_int(kind),
              ctypes.c_double(scale))


def loss_seed(lat, f, target_u, weight=None, kind=LOSS_VEC, scale=1.0):
    out = np.zeros(lat.shape + (lat.q,))
    w = _f64(weight) if weight is not None else None
    lib().orc_loss_seed(*lat.args(), _p(_f64(f)), _p(_f64(target_u)), _p(w),
                        ctypes.c_int(kind), ctypes.c_double(scale), _p(out))
    return out


def collide_adj(lat, tau, f, fsbar):
    """(dL/df, dL/dtau contribution) through one collision pass at state f."""
    fbar = np.zeros(lat.shape + (lat.q,))
    dtau = ctypes.c_double(0.0)
    lib().orc_collide_adj(*lat.args(), ctypes.c_double(tau), _p(_f64(f)), _p(_f64(fsbar)),
                          _p(fbar), ctypes.byref(dtau))
    return fbar, dtau.value


def stream_adj(lat, gbar):
    fsbar = np.zeros(lat.shape + (lat.q,))
    lib().orc_stream_adj(*lat.args(), _p(_f64(gbar)), _p(fsbar))
    return fsbar


def zouhe_adj(lat, gbar, g=None, rho_in=None):
    """(gbar after the Zou-He transpose, d/drho_in, d/drho_out) per face node.
    A velocity inlet also needs the completed state g and the inlet values."""
    gbar = _f64(gbar).copy()
    din = np.zeros((lat.nz, lat.ny))
    dout = np.zeros((lat.nz, lat.ny))
    gp = _p(_f64(g)) if g is not None else None
    rp = _p(lat.face(rho_in)) if rho_in is not None else None
    lib().orc_zouhe_adj(*lat.args(), gp, rp, _p(gbar), _p(din), _p(dout))
    return gbar, din, dout


def mrt_matrix():
    """The D2Q9 moment basis M (9 x 9) as the oracle builds it."""
    m = np.zeros((9, 9))
    lib().orc_mrt_matrix(_p(m))
    return m


def grad(lat, tau, rho_in, rho_out, f0, T, target_u, weight=None, kind=LOSS_VEC,
         scale=1.0, K=0, want_f0_bar=False, frames=1, stride=1):
    """Reverse-mode gradient of the loss after T steps.  frames > 1: the loss
    sums over the states after steps T - (frames - 1 - m) * stride, target_u
    holding one target per frame (frames, *shape, 3).

    Returns dict(loss, drho_in (nz, ny), drho_out (nz, ny), dtau[, df0])."""
    din = np.zeros((lat.nz, lat.ny))
    dout = np.zeros((lat.nz, lat.ny))
    dtau = ctypes.c_double(0.0)
    fb = np.zeros(lat.shape + (lat.q,)) if want_f0_bar else None
    w = _f64(weight) if weight is not None else None
    fn = lib().orc_grad
    fn.restype = ctypes.c_double
    L = fn(*lat.args(), ctypes.c_double(tau), _p(lat.face(rho_in)), _p(lat.face(rho_out)),
           _p(_f64(f0)), ctypes.c_int(T), ctypes.c_int(K), _p(_f64(target_u)), _p(w),
           ctypes.c_int(kind), ctypes.c_double(scale), ctypes.c_int(frames), ctypes.c_int(stride),
           _p(din), _p(dout), ctypes.byref(dtau), _p(fb))
    out = dict(loss=L, drho_in=din, drho_out=dout, dtau=dtau.value)
    if want_f0_bar:
        out["df0"] = fb
    return out


def loss_complex_step(lat, tau, rho_in, rho_out, f0, T, target_u, weight=None,
                      kind=LOSS_VEC, scale=1.0, dtau=0.0, drho_in=0.0, drho_out=0.0,
                      h=1e-30, frames=1, stride=1):
    """(loss, directional derivative) along (dtau, drho_in, drho_out) by the
    complex-step method: Im L(p + i h v) / h.  frames, stride: as in grad."""
    res = np.zeros(2)
    w = _f64(weight) if weight is not None else None
    lib().orc_run_loss_cs(*lat.args(), ctypes.c_double(tau), ctypes.c_double(h * dtau),
                          _p(lat.face(rho_in)), _p(lat.face(np.asarray(drho_in) * h)),
                          _p(lat.face(rho_out)), _p(lat.face(np.asarray(drho_out) * h)),
                          _p(_f64(f0)), ctypes.c_int(T), _p(_f64(target_u)), _p(w),
                          ctypes.c_int(kind), ctypes.c_double(scale), ctypes.c_int(frames),
                          ctypes.c_int(stride), _p(res))
    return res[0], res[1] / h


def set_threads(n):
    """Threads of the oracle's per-node loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def threads():
    return int(lib().orc_get_threads())


def velset(q):
    """(c (q, 3) int, w (q,), opp (q,)) exactly as the C oracle holds them."""
    c = np.zeros((q, 3), np.int32)
    w = np.zeros(q)
    opp = np.zeros(q, np.int32)
    ip = ctypes.POINTER(ctypes.c_int)
    lib().orc_velset_get(q, c.ctypes.data_as(ip), _p(w), opp.ctypes.data_as(ip))
    return c, w, opp


def jvp_steps(lat, tau, rho_in, rho_out, f0, v, T, h=1e-30):
    """(state after T steps, Jacobian of the T-step map applied to v), by the
    complex-step method on the populations."""
    fr = _f64(f0).copy()
    fi = _f64(v) * h
    lib().orc_run_cs(*lat.args(), ctypes.c_double(tau), _p(lat.face(rho_in)),
                     _p(lat.face(rho_out)), _p(fr), _p(fi), ctypes.c_int(T))
    return fr, fi / h
