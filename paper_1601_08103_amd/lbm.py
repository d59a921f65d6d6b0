"""Python binding of liblbm_lee.so: argument marshalling only, same names as the C ABI.

Every step of the computation runs in the HIP library; PyTorch only provides device memory
and the stream.  Importing works without a GPU, but loading the library fails loudly if it
has not been built (python -m paper_1601_08103_amd.build).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbm_lee.so")

LATTICES = {"D1Q3": 0, "D2Q5": 1, "D2Q9": 2, "D3Q7": 3, "D3Q9": 4, "D3Q13": 5, "D3Q19": 6,
            "D2Q5_DIA": 7, "D3Q7_DIA": 8, "D3Q27": 9}
STORAGES = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3, "i16": 4, "e3m12": 5}
ELEM_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2, "i16": 2, "e3m12": 2}
TUNE = {"nt_store": 1, "nt_load": 2, "persistent": 4, "full_rest": 8, "closure_stream": 16, "in_place": 32,
        "tb_segment_8": 64, "tb_segment_16": 128, "tb_segment_32": 192, "net_one_block": 256}
VARIANTS = {"auto": 0, "generic": 1, "dpp": 2, "lds": 3, "dpp2": 4, "tb2": 5, "tb3": 6, "open2d": 7, "resident": 8}
BCS = {"periodic": 0, "zero": 1, "copy": 2, "sponge": 3, "mlp": 4}

LBM_OK = 0


class LbmError(RuntimeError):
    def __init__(self, func, status, msg):
        super().__init__(f"{func} failed with status {status}: {msg}")
        self.status = status


class lbm_lee_desc(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("storage", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
                ("tau", ctypes.c_double), ("variant", ctypes.c_int32), ("tune", ctypes.c_int32),
                ("store_scale", ctypes.c_double), ("bc", ctypes.c_int32), ("sponge_width", ctypes.c_int32),
                ("sponge_sigma", ctypes.c_double)]


class lbm_lee_scaling(ctypes.Structure):
    _fields_ = [("rho_star", ctypes.c_double), ("theta_star", ctypes.c_double), ("u_star", ctypes.c_double),
                ("x_star", ctypes.c_double), ("t_star", ctypes.c_double)]


class lbm_lattice_info(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("Q", ctypes.c_int32), ("c", (ctypes.c_int32 * 3) * 27),
                ("fstar", ctypes.c_double * 27), ("beta", ctypes.c_double * 27),
                ("rho0", ctypes.c_double), ("theta0", ctypes.c_double), ("gamma", ctypes.c_double),
                ("a1", ctypes.c_double), ("a2", ctypes.c_double), ("b", ctypes.c_double),
                ("c1", ctypes.c_double), ("c2", ctypes.c_double), ("name", ctypes.c_char * 16)]


# symbol -> (restype, argtypes)
_VP = ctypes.c_void_p
_DESC_P = ctypes.POINTER(lbm_lee_desc)
SIGNATURES = {
    "lbm_lee_lattice_info": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(lbm_lattice_info)]),
    "lbm_lee_dimensional_scaling": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                                     ctypes.c_double, ctypes.POINTER(lbm_lee_scaling)]),
    "lbm_lee_dimensional_steps": (ctypes.c_int32, [ctypes.POINTER(lbm_lee_scaling), ctypes.c_double, ctypes.c_double,
                                                   ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                                   ctypes.POINTER(ctypes.c_double)]),
    "lbm_lee_state_bytes": (ctypes.c_size_t, [_DESC_P]),
    "lbm_lee_scratch_bytes": (ctypes.c_size_t, [_DESC_P]),
    "lbm_lee_bytes_per_update": (ctypes.c_double, [_DESC_P]),
    "lbm_lee_collision_constants": (ctypes.c_int, [_DESC_P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_lee_init": (ctypes.c_int32, [_DESC_P, _VP, _VP, ctypes.c_size_t, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP,
                                      ctypes.POINTER(_VP)]),
    "lbm_lee_reinit": (ctypes.c_int32, [_VP, _VP, _VP, _VP, _VP]),
    "lbm_lee_step": (ctypes.c_int32, [_VP, ctypes.c_int64, _VP]),
    "lbm_lee_reinit_region": (ctypes.c_int32, [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                               _VP, _VP, _VP, _VP]),
    "lbm_lee_moments_region": (ctypes.c_int32, [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                                _VP, _VP, _VP, _VP, ctypes.c_int32, _VP]),
    "lbm_lee_moments": (ctypes.c_int32, [_VP, _VP, _VP, _VP, _VP, ctypes.c_int32, _VP]),
    "lbm_lee_l2_energy": (ctypes.c_int32, [_VP, ctypes.POINTER(ctypes.c_double), _VP]),
    "lbm_lee_error_norms": (ctypes.c_int32, [_VP, _VP, _VP, ctypes.POINTER(ctypes.c_double), _VP]),
    "lbm_lee_export_f64": (ctypes.c_int32, [_VP, _VP, _VP]),
    "lbm_lee_import_f64": (ctypes.c_int32, [_VP, _VP, ctypes.c_int64, _VP]),
    "lbm_lee_current": (ctypes.c_int32, [_VP, ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_int64)]),
    "lbm_lee_store_scale": (ctypes.c_double, [_VP]),
    "lbm_lee_resolved_variant": (ctypes.c_int32, [_VP]),
    "lbm_lee_destroy": (None, [_VP]),
    "lbm_lee_device_copy": (ctypes.c_int32, [_VP, _VP, ctypes.c_size_t, _VP]),
    "lbm_lee_ghost_bytes": (ctypes.c_size_t, [_DESC_P]),
    "lbm_lee_set_closure": (ctypes.c_int32, [_VP, _VP, _VP, ctypes.c_size_t]),
    "lbm_nrbc_dims": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "lbm_nrbc_face_nodes": (ctypes.c_int64, [_DESC_P]),
    "lbm_nrbc_forward": (ctypes.c_int32, [ctypes.c_int32, _VP, _VP, ctypes.c_int64, _VP, _VP]),
    "lbm_nrbc_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int64]),
    "lbm_nrbc_loss_grad": (ctypes.c_int32, [ctypes.c_int32, _VP, _VP, _VP, ctypes.c_int64, _VP, _VP, _VP,
                                            ctypes.c_size_t, _VP]),
    "lbm_nrbc_adam": (ctypes.c_int32, [ctypes.c_int64, _VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float, ctypes.c_float, _VP]),
    "lbm_nrbc_gather": (ctypes.c_int32, [_VP, ctypes.POINTER(ctypes.c_int64), _DESC_P, _VP, ctypes.c_int64, _VP,
                                         ctypes.c_int64, _VP, _VP]),
    "lbm_lee_compare_fields": (ctypes.c_int32, [_VP, ctypes.POINTER(ctypes.c_int64), _VP,
                                                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                                ctypes.POINTER(ctypes.c_double), _VP, ctypes.c_size_t, _VP]),
    "lbm_lee_compare_fields_static": (ctypes.c_int32, [_VP, ctypes.POINTER(ctypes.c_int64), _VP,
                                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                                       ctypes.POINTER(ctypes.c_double), _VP]),
    "lbm_lee_last_error": (ctypes.c_char_p, []),
    "lbm_lee_version": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load the in-tree HIP library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1601_08103_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(name, status):
    if status != LBM_OK:
        raise LbmError(name, status, load().lbm_lee_last_error().decode())


def make_desc(lattice: str, storage: str, shape, tau: float = 0.5, variant: str = "auto",
              store_scale: float = 0.0, tune: int = 0, bc: str = "periodic", sponge_width: int = 0,
              sponge_sigma: float = 0.0) -> lbm_lee_desc:
    """Descriptor for a spatial shape given in C order ((nz, ny, nx), (ny, nx) or (nx,))."""
    dims = list(reversed([int(s) for s in shape])) + [1] * (3 - len(shape))
    d = lbm_lee_desc()
    d.lattice = LATTICES[lattice]
    d.storage = STORAGES[storage]
    for a in range(3):
        d.n[a] = dims[a]
    d.tau = float(tau)
    d.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    d.tune = int(tune)
    d.store_scale = float(store_scale)
    d.bc = BCS[bc]
    d.sponge_width = int(sponge_width)
    d.sponge_sigma = float(sponge_sigma)
    return d


# ------------------------------------------------------------------ thin wrappers (same names)
def lbm_lee_lattice_info(lattice: str) -> dict:
    info = lbm_lattice_info()
    _check("lbm_lee_lattice_info", load().lbm_lee_lattice_info(LATTICES[lattice], ctypes.byref(info)))
    Q = info.Q
    return dict(D=info.D, Q=Q, c=np.array([[info.c[i][a] for a in range(3)] for i in range(Q)], dtype=np.int64),
                fstar=np.array(info.fstar[:Q]), beta=np.array(info.beta[:Q]), rho0=info.rho0,
                theta0=info.theta0, gamma=info.gamma, a1=info.a1, a2=info.a2, b=info.b, c1=info.c1, c2=info.c2,
                name=info.name.decode())


def lbm_lee_dimensional_scaling(lattice: str, rho0_dim: float, theta0_dim: float, x_star: float = 1.0):
    s = lbm_lee_scaling()
    _check("lbm_lee_dimensional_scaling", load().lbm_lee_dimensional_scaling(LATTICES[lattice], float(rho0_dim),
                                                                             float(theta0_dim), float(x_star),
                                                                             ctypes.byref(s)))
    return s


def lbm_lee_dimensional_steps(scaling, t_dim: float, dt: float):
    """(nsteps, t_end, offset) for a dimensional end time with non-dimensional step dt."""
    n = ctypes.c_int64()
    te = ctypes.c_double()
    off = ctypes.c_double()
    _check("lbm_lee_dimensional_steps", load().lbm_lee_dimensional_steps(ctypes.byref(scaling), float(t_dim), float(dt),
                                                                         ctypes.byref(n), ctypes.byref(te),
                                                                         ctypes.byref(off)))
    return int(n.value), float(te.value), float(off.value)


def lbm_lee_state_bytes(desc) -> int:
    return int(load().lbm_lee_state_bytes(ctypes.byref(desc)))


def lbm_lee_scratch_bytes(desc) -> int:
    return int(load().lbm_lee_scratch_bytes(ctypes.byref(desc)))


def lbm_lee_bytes_per_update(desc) -> float:
    return float(load().lbm_lee_bytes_per_update(ctypes.byref(desc)))


def lbm_lee_collision_constants(desc):
    """(H (4, 4), WB (4, 4), keep): the step kernels' folded collision constants in FP64."""
    H = np.zeros(16)
    WB = np.zeros(16)
    keep = ctypes.c_double(0.0)
    _check("lbm_lee_collision_constants",
           load().lbm_lee_collision_constants(ctypes.byref(desc), H.ctypes.data, WB.ctypes.data, ctypes.byref(keep)))
    return H.reshape(4, 4), WB.reshape(4, 4), keep.value


def lbm_lee_init(desc, pop_a, pop_b, bytes_each, rho, u, theta, scratch, scratch_bytes, stream) -> int:
    h = _VP()
    _check("lbm_lee_init", load().lbm_lee_init(ctypes.byref(desc), pop_a, pop_b, bytes_each, rho, u, theta, scratch,
                                               scratch_bytes, stream, ctypes.byref(h)))
    return h.value


def lbm_lee_reinit(h, rho, u, theta, stream):
    _check("lbm_lee_reinit", load().lbm_lee_reinit(h, rho, u, theta, stream))


def lbm_lee_reinit_region(h, origin, n_sub, rho, u, theta, stream):
    _check("lbm_lee_reinit_region", load().lbm_lee_reinit_region(h, _i64x3(origin), _i64x3(n_sub), rho, u, theta,
                                                                 stream))


def lbm_lee_moments_region(h, origin, n_sub, p, u, rho, theta, out_is_f64, stream):
    _check("lbm_lee_moments_region", load().lbm_lee_moments_region(h, _i64x3(origin), _i64x3(n_sub), p, u, rho, theta,
                                                                   int(out_is_f64), stream))


def lbm_lee_step(h, nsteps, stream):
    _check("lbm_lee_step", load().lbm_lee_step(h, int(nsteps), stream))


def lbm_lee_moments(h, p, u, rho, theta, out_is_f64, stream):
    _check("lbm_lee_moments", load().lbm_lee_moments(h, p, u, rho, theta, int(out_is_f64), stream))


def lbm_lee_l2_energy(h, stream):
    out = (ctypes.c_double * 2)()
    _check("lbm_lee_l2_energy", load().lbm_lee_l2_energy(h, out, stream))
    return float(out[0]), float(out[1])


def lbm_lee_error_norms(h, ref_p, ref_u, stream):
    out = (ctypes.c_double * 6)()
    _check("lbm_lee_error_norms", load().lbm_lee_error_norms(h, ref_p, ref_u, out, stream))
    return [float(v) for v in out]


def lbm_lee_export_f64(h, g, stream):
    _check("lbm_lee_export_f64", load().lbm_lee_export_f64(h, g, stream))


def lbm_lee_import_f64(h, g, steps_done, stream):
    _check("lbm_lee_import_f64", load().lbm_lee_import_f64(h, g, int(steps_done), stream))


def lbm_lee_current(h):
    p = _VP()
    n = ctypes.c_int64()
    _check("lbm_lee_current", load().lbm_lee_current(h, ctypes.byref(p), ctypes.byref(n)))
    return p.value, int(n.value)


def lbm_lee_store_scale(h) -> float:
    return float(load().lbm_lee_store_scale(h))


def lbm_lee_resolved_variant(h) -> int:
    return int(load().lbm_lee_resolved_variant(h))


def lbm_lee_destroy(h):
    load().lbm_lee_destroy(h)


def lbm_lee_device_copy(dst, src, nbytes, stream):
    _check("lbm_lee_device_copy", load().lbm_lee_device_copy(dst, src, int(nbytes), stream))


def lbm_lee_ghost_bytes(desc) -> int:
    return int(load().lbm_lee_ghost_bytes(ctypes.byref(desc)))


def lbm_lee_set_closure(h, params, ghost, ghost_bytes):
    _check("lbm_lee_set_closure", load().lbm_lee_set_closure(h, params, ghost, ghost_bytes))


def lbm_nrbc_dims(lattice: str) -> dict:
    d = (ctypes.c_int32 * 4)()
    _check("lbm_nrbc_dims", load().lbm_nrbc_dims(LATTICES[lattice], d))
    return dict(n_in=d[0], n_out=d[1], hidden=d[2], n_params=d[3])


def lbm_nrbc_face_nodes(desc) -> int:
    return int(load().lbm_nrbc_face_nodes(ctypes.byref(desc)))


def lbm_nrbc_forward(lattice, params, strips, count, out, stream):
    _check("lbm_nrbc_forward", load().lbm_nrbc_forward(LATTICES[lattice], params, strips, int(count), out, stream))


def lbm_nrbc_workspace_bytes(lattice, count) -> int:
    return int(load().lbm_nrbc_workspace_bytes(LATTICES[lattice], int(count)))


def lbm_nrbc_loss_grad(lattice, params, strips, targets, count, grad, loss, workspace, workspace_bytes, stream):
    _check("lbm_nrbc_loss_grad", load().lbm_nrbc_loss_grad(LATTICES[lattice], params, strips, targets, int(count),
                                                           grad, loss, workspace, int(workspace_bytes), stream))


def lbm_nrbc_adam(n, params, grad, m, v, t, lr, beta1, beta2, eps, stream):
    _check("lbm_nrbc_adam", load().lbm_nrbc_adam(int(n), params, grad, m, v, int(t), float(lr), float(beta1),
                                                 float(beta2), float(eps), stream))


def _i64x3(v):
    return (ctypes.c_int64 * 3)(*[int(x) for x in v])


def lbm_nrbc_gather(outer, origin, inner_desc, node_ids, count, strips, strip_stride, targets, stream):
    _check("lbm_nrbc_gather", load().lbm_nrbc_gather(outer, _i64x3(origin), ctypes.byref(inner_desc), node_ids,
                                                     int(count), strips, int(strip_stride), targets, stream))


def lbm_lee_compare_fields(a, n_a, b, n_b, origin, scratch, scratch_bytes, stream):
    out = (ctypes.c_double * 3)()
    _check("lbm_lee_compare_fields", load().lbm_lee_compare_fields(a, _i64x3(n_a), b, _i64x3(n_b), _i64x3(origin),
                                                                   out, scratch, int(scratch_bytes), stream))
    return [float(v) for v in out]


def lbm_lee_compare_fields_static(a, n_a, b, n_b, origin, stream):
    out = (ctypes.c_double * 3)()
    _check("lbm_lee_compare_fields_static", load().lbm_lee_compare_fields_static(a, _i64x3(n_a), b, _i64x3(n_b),
                                                                                 _i64x3(origin), out, stream))
    return [float(v) for v in out]


def lbm_lee_version() -> str:
    return load().lbm_lee_version().decode()


# ------------------------------------------------------------------ convenience object
class Solver:
    """Owns torch device buffers for one solver handle; every method is one C-ABI call."""

    def __init__(self, lattice: str, storage: str, shape, rho, u, theta, tau: float = 0.5, variant: str = "auto",
                 store_scale: float = 0.0, tune: int = 0, bc: str = "periodic", sponge_width: int = 0,
                 sponge_sigma: float = 0.0, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the LEE-LBM solver needs a GPU")
        self.torch = torch
        self.lattice, self.storage = lattice, storage
        self.shape = tuple(int(s) for s in shape)
        self.info = lbm_lee_lattice_info(lattice)
        self.D, self.Q = self.info["D"], self.info["Q"]
        if len(self.shape) != self.D:
            raise ValueError(f"{lattice} needs a {self.D}D shape, got {self.shape}")
        self.N = int(np.prod(self.shape))
        self.desc = make_desc(lattice, storage, self.shape, tau, variant, store_scale, tune, bc, sponge_width,
                              sponge_sigma)
        self.state_bytes = lbm_lee_state_bytes(self.desc)
        if self.state_bytes == 0:
            load()
            raise LbmError("lbm_lee_state_bytes", -1, load().lbm_lee_last_error().decode())
        self.scratch_bytes = lbm_lee_scratch_bytes(self.desc)
        dev = torch.device("cuda")
        self.pop_a = torch.empty(self.state_bytes, dtype=torch.uint8, device=dev)
        in_place = bool(int(tune) & TUNE["in_place"])
        self.pop_b = None if in_place else torch.empty(self.state_bytes, dtype=torch.uint8, device=dev)
        self.scratch = torch.empty(self.scratch_bytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if rho is None and u is None and theta is None:  # the state at rest
            ptrs, self._keep = (None, None, None), ()
        else:
            self._keep = self._fields(rho, u, theta)  # the init kernel may still be reading them
            ptrs = tuple(a.data_ptr() for a in self._keep)
        self.h = lbm_lee_init(self.desc, self.pop_a.data_ptr(),
                              self.pop_b.data_ptr() if self.pop_b is not None else None, self.state_bytes, *ptrs,
                              self.scratch.data_ptr(), self.scratch_bytes, self.stream.cuda_stream)

    def _fields(self, rho, u, theta):
        t = self.torch
        dev = t.device("cuda")
        def as_dev(a, n):
            a = t.as_tensor(a, dtype=t.float64).to(dev).contiguous()
            if a.numel() != n:
                raise ValueError(f"field has {a.numel()} values, expected {n}")
            return a
        return as_dev(rho, self.N), as_dev(u, self.D * self.N), as_dev(theta, self.N)

    @property
    def s(self):
        return self.stream.cuda_stream

    def reinit(self, rho, u, theta):
        self._keep = self._fields(rho, u, theta)
        lbm_lee_reinit(self.h, self._keep[0].data_ptr(), self._keep[1].data_ptr(), self._keep[2].data_ptr(), self.s)

    def step(self, n: int = 1):
        lbm_lee_step(self.h, n, self.s)

    def reinit_region(self, origin_xyz, sub_shape, rho, u, theta):
        """Equilibrium of fields given on a sub-box (C-order shape sub_shape at cell offset
        origin_xyz = (x, y, z)), the state at rest elsewhere."""
        t = self.torch
        sub = tuple(int(v) for v in sub_shape)
        n = int(np.prod(sub))
        def dev(a, m):
            a = t.as_tensor(a, dtype=t.float64).to("cuda").contiguous()
            if a.numel() != m:
                raise ValueError("field size does not match the sub-box")
            return a
        self._keep = (dev(rho, n), dev(u, self.D * n), dev(theta, n))
        dims = list(reversed(sub)) + [1] * (3 - len(sub))
        org = list(origin_xyz) + [0] * (3 - len(origin_xyz))
        lbm_lee_reinit_region(self.h, org, dims, self._keep[0].data_ptr(), self._keep[1].data_ptr(),
                              self._keep[2].data_ptr(), self.s)

    def moments_region(self, origin_xyz, sub_shape, f64: bool = True) -> dict:
        t = self.torch
        sub = tuple(int(v) for v in sub_shape)
        n = int(np.prod(sub))
        dt = t.float64 if f64 else t.float32
        out = {k: t.empty(n, dtype=dt, device="cuda") for k in ("p", "rho", "theta")}
        out["u"] = t.empty(self.D * n, dtype=dt, device="cuda")
        dims = list(reversed(sub)) + [1] * (3 - len(sub))
        org = list(origin_xyz) + [0] * (3 - len(origin_xyz))
        lbm_lee_moments_region(self.h, org, dims, out["p"].data_ptr(), out["u"].data_ptr(), out["rho"].data_ptr(),
                               out["theta"].data_ptr(), int(f64), self.s)
        res = {k: v.view(sub) for k, v in out.items() if k != "u"}
        res["u"] = out["u"].view((self.D,) + sub)
        return res

    def moments(self, f64: bool = True) -> dict:
        t = self.torch
        dt = t.float64 if f64 else t.float32
        out = {k: t.empty(self.N, dtype=dt, device="cuda") for k in ("p", "rho", "theta")}
        out["u"] = t.empty(self.D * self.N, dtype=dt, device="cuda")
        lbm_lee_moments(self.h, out["p"].data_ptr(), out["u"].data_ptr(), out["rho"].data_ptr(),
                        out["theta"].data_ptr(), int(f64), self.s)
        res = {k: v.view(self.shape) for k, v in out.items() if k != "u"}
        res["u"] = out["u"].view((self.D,) + self.shape)
        return res

    def l2_energy(self):
        return lbm_lee_l2_energy(self.h, self.s)

    def error_norms(self, ref_p, ref_u=None):
        t = self.torch
        rp = t.as_tensor(ref_p, dtype=t.float64).to("cuda").contiguous()
        ru = None if ref_u is None else t.as_tensor(ref_u, dtype=t.float64).to("cuda").contiguous()
        return lbm_lee_error_norms(self.h, rp.data_ptr(), None if ru is None else ru.data_ptr(), self.s)

    def export_f64(self):
        t = self.torch
        g = t.empty((self.Q,) + self.shape, dtype=t.float64, device="cuda")
        lbm_lee_export_f64(self.h, g.data_ptr(), self.s)
        return g

    def import_f64(self, g, steps_done: int = 0):
        t = self.torch
        gt = t.as_tensor(g, dtype=t.float64).to("cuda").contiguous()
        if gt.numel() != self.Q * self.N:
            raise ValueError("population array has the wrong size")
        lbm_lee_import_f64(self.h, gt.data_ptr(), steps_done, self.s)
        self._keep = (gt,)

    def current(self):
        return lbm_lee_current(self.h)

    def set_closure(self, params):
        """Attach closure-network parameters (FP32, device or host array) for LBM_BC_MLP."""
        t = self.torch
        self._net = t.as_tensor(params, dtype=t.float32).to("cuda").contiguous()
        nb = lbm_lee_ghost_bytes(self.desc)
        self._ghost = t.zeros(max(nb // 4, 1), dtype=t.float32, device="cuda")
        lbm_lee_set_closure(self.h, self._net.data_ptr(), self._ghost.data_ptr(), nb)

    @property
    def ghost(self):
        return self._ghost

    @property
    def store_scale(self) -> float:
        return lbm_lee_store_scale(self.h)

    @property
    def variant(self) -> str:
        v = lbm_lee_resolved_variant(self.h)
        return {val: key for key, val in VARIANTS.items()}[v]

    @property
    def bytes_per_update(self) -> float:
        return lbm_lee_bytes_per_update(self.desc)

    def close(self):
        if getattr(self, "h", None):
            lbm_lee_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
