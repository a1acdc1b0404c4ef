"""Thin ctypes binding of libnmr (the C ABI in include/nmr.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch supplies device memory and the stream.  Importing this
module does not load the library; ``lib()`` does, and raises if the HIP
library has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnmr.so")

PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
TRAIN_PHASES = ["s_epoch", "w_epoch", "s_elem_fwd", "s_elem_bwd"]
PHASES = ["dec_hidden", "dec_out", "cubature", "mass", "sums", "bwd_out", "bwd_hidden", "solve"]
# kernels of each phase, as rocprofv3 names them
PHASE_KERNELS = {"dec_hidden": "k_fwd_hidden", "dec_out": "k_fwd_out", "cubature": "k_cubature", "mass": "k_mass",
                 "sums": "k_sums", "bwd_out": "k_bwd_out", "bwd_hidden": "k_bwd_hidden", "solve": "k_solve"}
ACT = {"identity": 0, "tanh": 1, "elu": 2, "sin": 3}
STATUS = {0: "ok", -1: "arg", -2: "budget", -3: "oom", -4: "inverted", -5: "singular", -6: "nonfinite",
          -7: "device"}

_dp = C.POINTER(C.c_double)


class MlpDesc(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("widths", C.POINTER(C.c_int)), ("act", C.c_int),
                ("W", C.POINTER(_dp)), ("b", C.POINTER(_dp))]


class ProblemDesc(C.Structure):
    _fields_ = [("n_vertices", C.c_int), ("X", _dp), ("n_tets", C.c_int), ("tets", C.POINTER(C.c_int32)),
                ("pinned", C.POINTER(C.c_uint8)), ("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double),
                ("gravity", C.c_double * 3), ("dt", C.c_double), ("n_p", C.c_int), ("U", _dp),
                ("decoder", C.POINTER(MlpDesc)), ("shared_decoder", C.c_void_p), ("n_cub", C.c_int),
                ("cub_ids", C.POINTER(C.c_int32)), ("cub_w", _dp), ("wnet", C.POINTER(MlpDesc)),
                ("wnet_scale", C.c_double), ("r0", _dp), ("rdot0", _dp), ("newton_path", C.c_int),
                ("trimmed", C.c_int), ("fd_h", C.c_double)]


class TileChoice(C.Structure):
    _fields_ = [("forward", C.c_int), ("m_in", C.c_int), ("m_out", C.c_int), ("cols", C.c_int),
                ("n_inst", C.c_int), ("prec", C.c_int), ("ib", C.c_int), ("mr", C.c_int), ("jet_groups", C.c_int),
                ("us", C.c_float)]


TILING = {"rule": 0, "autotune": 1, "force": 2}


class TrainDesc(C.Structure):
    _fields_ = [("n_poses", C.c_int), ("poses", _dp), ("c_max", C.c_int), ("n_c0", C.c_int),
                ("c0", C.POINTER(C.c_int32)), ("K", C.c_int), ("epochs", C.c_int), ("lr", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double), ("wnet", C.POINTER(MlpDesc)),
                ("wnet_scale", C.c_double), ("snet", _dp), ("pose_chunk", C.c_int)]


class NmrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_LIB = None


def lib():
    """Load libnmr.so; raise if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run paper_2102_11026_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp, ip, i = C.c_void_p, C.POINTER(C.c_int), C.c_int
        sig = {
            "nmr_create": (i, [i, vp, C.c_size_t, C.POINTER(vp)]),
            "nmr_destroy": (i, [vp]),
            "nmr_last_error": (C.c_char_p, []),
            "nmr_decoder_create": (i, [vp, C.POINTER(MlpDesc), i, C.POINTER(vp)]),
            "nmr_decoder_destroy": (i, [vp]),
            "nmr_instance_create": (i, [vp, C.POINTER(ProblemDesc), i, C.POINTER(vp)]),
            "nmr_instance_destroy": (i, [vp]),
            "nmr_instance_bytes": (i, [vp, C.POINTER(C.c_size_t)]),
            "nmr_instance_newton_path": (i, [vp, C.POINTER(C.c_int)]),
            "nmr_instance_get_state": (i, [vp, _dp, _dp, vp]),
            "nmr_instance_set_state": (i, [vp, _dp, _dp]),
            "nmr_instance_status": (i, [vp]),
            "nmr_instance_get_frame": (i, [vp, vp]),
            "nmr_instance_frame_ptr": (i, [vp, C.POINTER(vp)]),
            "decoder_jacobian_hessian": (i, [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
            "cubature_force_stiffness": (i, [vp, vp, vp, vp, vp, vp, vp]),
            "cubature_force_stiffness_noalloc": (i, [vp, vp, vp, vp, vp, vp, vp]),
            "reduced_newton_system": (i, [vp, vp, vp, vp]),
            "reduced_newton_step": (i, [vp, i, _dp]),
            "step_many": (i, [vp, C.POINTER(vp), i, i, i, ip, C.POINTER(C.c_float)]),
            "nmr_time_phase": (i, [vp, i, i, C.POINTER(C.c_float)]),
            "nmr_set_tiling": (i, [vp, i, i, i]),
            "nmr_tiling_table": (i, [vp, C.POINTER(TileChoice), i, ip]),
            "nmr_coupled_create": (i, [vp, vp, i, C.POINTER(vp), C.POINTER(C.c_int32), i, C.c_double,
                                       C.POINTER(vp)]),
            "nmr_coupled_destroy": (i, [vp]),
            "nmr_coupled_step": (i, [vp, i, i, ip, C.POINTER(C.c_float)]),
            "nmr_pool_create": (i, [vp, i, C.POINTER(vp)]),
            "nmr_pool_destroy": (i, [vp]),
            "nmr_pool_attach": (i, [vp, vp, ip]),
            "nmr_pool_detach": (i, [vp, i]),
            "nmr_pool_step": (i, [vp, i, ip, C.POINTER(C.c_float)]),
            "nmr_element_forces": (i, [vp, vp, vp, vp, vp]),
            "nmr_trainer_create": (i, [vp, C.POINTER(TrainDesc), C.POINTER(vp)]),
            "nmr_trainer_destroy": (i, [vp]),
            "nmr_trainer_run": (i, [vp, i, _dp, _dp, ip, C.POINTER(C.c_float)]),
            "nmr_trainer_get": (i, [vp, ip, C.POINTER(C.c_int32), _dp, _dp]),
            "nmr_trainer_pose": (i, [vp, i, _dp, _dp, _dp]),
            "nmr_trainer_time_phase": (i, [vp, i, i, C.POINTER(C.c_float)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _check(rc: int):
    if rc != 0:
        raise NmrError(rc, lib().nmr_last_error().decode())


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class _Mlp:
    """Keeps the host arrays of an MLP description alive."""

    def __init__(self, Ws, bs, act: str):
        self.W = [np.ascontiguousarray(W, dtype=np.float64) for W in Ws]
        self.b = [np.ascontiguousarray(b, dtype=np.float64) for b in bs]
        widths = [self.W[0].shape[1]] + [W.shape[0] for W in self.W]
        self.widths = (C.c_int * len(widths))(*widths)
        self.Wp = (_dp * len(self.W))(*[W.ctypes.data_as(_dp) for W in self.W])
        self.bp = (_dp * len(self.b))(*[b.ctypes.data_as(_dp) for b in self.b])
        self.desc = MlpDesc(len(self.W), self.widths, ACT[act], self.Wp, self.bp)


class Context:
    def __init__(self, device: int = 0, stream=None, budget_bytes: int = 0):
        import torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        _check(lib().nmr_create(device, C.c_void_p(stream.cuda_stream), budget_bytes, C.byref(h)))
        self.h = h

    def set_tiling(self, mode: str = "rule", ib: int = 1, mr: int = 1):
        """Tile choice of batched hidden-layer launches: "rule", "autotune" or
        "force" (ib instances per block, mr 16-row tiles per wave)."""
        _check(lib().nmr_set_tiling(self.h, TILING[mode], ib, mr))

    def tiling_table(self) -> list:
        """The autotuned choices so far, as dicts."""
        cap = 256
        buf = (TileChoice * cap)()
        n = C.c_int()
        _check(lib().nmr_tiling_table(self.h, buf, cap, C.byref(n)))
        names = [f[0] for f in TileChoice._fields_]
        return [{k: getattr(buf[j], k) for k in names} for j in range(n.value)]

    def close(self):
        if self.h:
            _check(lib().nmr_destroy(self.h))
            self.h = None


class Decoder:
    """A device decoder shared by several instances."""

    def __init__(self, ctx: Context, weights, biases, act: str, prec: str = "fp32"):
        m = _Mlp(weights, biases, act)
        h = C.c_void_p()
        _check(lib().nmr_decoder_create(ctx.h, C.byref(m.desc), PREC[prec], C.byref(h)))
        self.h, self.ctx, self.prec = h, ctx, prec

    def close(self):
        if self.h:
            _check(lib().nmr_decoder_destroy(self.h))
            self.h = None


class Instance:
    def __init__(self, ctx: Context, prob, prec: str = "fp32", shared: Optional[Decoder] = None,
                 path: str = "auto"):
        import torch
        self.ctx, self.prob, self.prec = ctx, prob, prec
        self.N, self.n_p, self.n_q, self.R = prob.N, prob.n_p, prob.n_q, prob.R
        self.n_cub = int(prob.cub_ids.size)
        self.rdtype = torch.float64 if prec == "fp64" else torch.float32
        self.dev = torch.device("cuda", ctx.device)
        keep = []
        X = np.ascontiguousarray(prob.X, np.float64)
        T = np.ascontiguousarray(prob.tets, np.int32)
        pin = np.ascontiguousarray(prob.pinned, np.uint8)
        U = np.ascontiguousarray(prob.U, np.float64)
        ids = np.ascontiguousarray(prob.cub_ids, np.int32)
        r0 = np.ascontiguousarray(prob.r0, np.float64)
        rd0 = np.ascontiguousarray(prob.rdot0, np.float64)
        keep += [X, T, pin, U, ids, r0, rd0]
        d = ProblemDesc()
        d.n_vertices, d.X = prob.n, X.ctypes.data_as(_dp)
        d.n_tets, d.tets = T.shape[0], T.ctypes.data_as(C.POINTER(C.c_int32))
        d.pinned = pin.ctypes.data_as(C.POINTER(C.c_uint8))
        d.E, d.nu, d.rho = prob.E, prob.nu, prob.rho
        d.gravity = (C.c_double * 3)(*prob.gravity)
        d.dt = prob.dt
        d.n_p = prob.n_p
        d.U = U.ctypes.data_as(_dp) if prob.n_p else None
        if shared is None:
            dm = _Mlp(prob.weights, prob.biases, prob.act)
            keep.append(dm)
            d.decoder = C.pointer(dm.desc)
            d.shared_decoder = None
        else:
            d.decoder = None
            d.shared_decoder = shared.h
        d.n_cub, d.cub_ids = ids.size, ids.ctypes.data_as(C.POINTER(C.c_int32))
        if prob.cub_w is not None:
            w = np.ascontiguousarray(prob.cub_w, np.float64)
            keep.append(w)
            d.cub_w = w.ctypes.data_as(_dp)
            d.wnet = None
        else:
            d.cub_w = None
            wm = _Mlp(prob.wnet_weights, prob.wnet_biases, "identity")
            keep.append(wm)
            d.wnet = C.pointer(wm.desc)
        d.wnet_scale = prob.wnet_scale
        d.r0, d.rdot0 = r0.ctypes.data_as(_dp), rd0.ctypes.data_as(_dp)
        d.newton_path = {"auto": 0, "direct": 1}[path]
        d.trimmed = {"full": 0, "trimmed": 1}[getattr(prob, "formulation", "full")]
        d.fd_h = float(getattr(prob, "fd_h", 0.0) or 0.0)
        h = C.c_void_p()
        _check(lib().nmr_instance_create(ctx.h, C.byref(d), PREC[prec], C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            _check(lib().nmr_instance_destroy(self.h))
            self.h = None

    @property
    def nbytes(self) -> int:
        b = C.c_size_t()
        _check(lib().nmr_instance_bytes(self.h, C.byref(b)))
        return b.value

    @property
    def gram(self) -> bool:
        """True if the instance runs the Gram-folded Newton path."""
        v = C.c_int()
        _check(lib().nmr_instance_newton_path(self.h, C.byref(v)))
        return v.value == 0

    # -- state ---------------------------------------------------------------
    def get_state(self, with_u: bool = False):
        r = np.zeros(self.R)
        rd = np.zeros(self.R)
        u = np.zeros(self.N, dtype=np.float64 if self.prec == "fp64" else np.float32) if with_u else None
        _check(lib().nmr_instance_get_state(self.h, r.ctypes.data_as(_dp), rd.ctypes.data_as(_dp),
                                            None if u is None else u.ctypes.data))
        return (r, rd, u) if with_u else (r, rd)

    def get_frame(self):
        """The frame buffer (host copy): u of the state the last step started
        from, or of the current state after get_state(with_u=True)."""
        u = np.zeros(self.N, dtype=np.float64 if self.prec == "fp64" else np.float32)
        _check(lib().nmr_instance_get_frame(self.h, u.ctypes.data))
        return u

    def frame_ptr(self) -> int:
        """Device address of the frame buffer (N reals)."""
        p = C.c_void_p()
        _check(lib().nmr_instance_frame_ptr(self.h, C.byref(p)))
        return p.value

    def set_state(self, r, rdot):
        r = np.ascontiguousarray(r, np.float64)
        rd = np.ascontiguousarray(rdot, np.float64)
        _check(lib().nmr_instance_set_state(self.h, r.ctypes.data_as(_dp), rd.ctypes.data_as(_dp)))

    def status(self) -> int:
        return lib().nmr_instance_status(self.h)

    # -- hot path --------------------------------------------------------------
    def step(self, n_iters: int, resid: bool = True):
        """One implicit-Euler step; returns ||phi|| per Newton iteration if resid."""
        if resid:
            out = np.zeros(n_iters)
            _check(lib().reduced_newton_step(self.h, n_iters, out.ctypes.data_as(_dp)))
            return out
        _check(lib().reduced_newton_step(self.h, n_iters, None))
        return None

    def decoder_jacobian_hessian(self, q, dq, qdot, a=None):
        import torch
        f64 = dict(dtype=torch.float64, device=self.dev)
        rt = dict(dtype=self.rdtype, device=self.dev)
        q, dq, qdot = (torch.as_tensor(np.asarray(x, np.float64), **f64).contiguous() for x in (q, dq, qdot))
        out = dict(u=torch.empty(self.N, **rt), J=torch.empty(self.N, self.n_q, **rt),
                   dJ=torch.empty(self.N, self.n_q, **rt), Hdd=torch.empty(self.N, **rt))
        B = JTa = at = None
        if a is not None:
            at = torch.as_tensor(np.asarray(a), **rt).contiguous() if not torch.is_tensor(a) else a.to(**rt).contiguous()
            B = torch.empty(self.n_q, self.n_q, **f64)
            JTa = torch.empty(self.n_q, **f64)
        torch.cuda.synchronize(self.dev)
        _check(lib().decoder_jacobian_hessian(self.h, _ptr(q), _ptr(dq), _ptr(qdot), _ptr(at), _ptr(out["u"]),
                                              _ptr(out["J"]), _ptr(out["dJ"]), _ptr(out["Hdd"]), _ptr(B),
                                              _ptr(JTa)))
        torch.cuda.synchronize(self.dev)
        if a is not None:
            out["B"], out["JTa"] = B, JTa
        return out

    def cubature_force_stiffness(self, u, Jt, w=None, want_fint: bool = True, noalloc: bool = False):
        """noalloc: call cubature_force_stiffness_noalloc (working memory in
        the library's static device array) instead."""
        import torch
        rt = dict(dtype=self.rdtype, device=self.dev)
        ut = torch.as_tensor(np.asarray(u), **rt).contiguous()
        Jtt = torch.as_tensor(np.asarray(Jt), **rt).contiguous()
        wt = None if w is None else torch.as_tensor(np.asarray(w), **rt).contiguous()
        fint = torch.empty(self.N, **rt) if want_fint else None
        fr = torch.empty(self.R, dtype=torch.float64, device=self.dev)
        Kr = torch.empty(self.R, self.R, dtype=torch.float64, device=self.dev)
        torch.cuda.synchronize(self.dev)
        fn = lib().cubature_force_stiffness_noalloc if noalloc else lib().cubature_force_stiffness
        _check(fn(self.h, _ptr(ut), _ptr(Jtt), _ptr(wt), _ptr(fint), _ptr(fr), _ptr(Kr)))
        torch.cuda.synchronize(self.dev)
        return dict(f_int=fint, fr=fr, Kr=Kr)

    def time_phase(self, phase: int, reps: int = 20) -> float:
        """Mean device microseconds of one phase of a Newton iteration."""
        us = C.c_float()
        _check(lib().nmr_time_phase(self.h, phase, reps, C.byref(us)))
        return us.value

    def newton_system(self, r):
        import torch
        rt = torch.as_tensor(np.asarray(r, np.float64), dtype=torch.float64, device=self.dev).contiguous()
        A = torch.empty(self.R, self.R, dtype=torch.float64, device=self.dev)
        phi = torch.empty(self.R, dtype=torch.float64, device=self.dev)
        torch.cuda.synchronize(self.dev)
        _check(lib().reduced_newton_system(self.h, _ptr(rt), _ptr(A), _ptr(phi)))
        torch.cuda.synchronize(self.dev)
        return A, phi

    def element_forces(self, r):
        """(F [n_tets, R], f [R], u [N]) at pose r, device FP64 tensors."""
        import torch
        f64 = dict(dtype=torch.float64, device=self.dev)
        rt = torch.as_tensor(np.asarray(r, np.float64), **f64).contiguous()
        F = torch.empty(int(self.prob.tets.shape[0]), self.R, **f64)
        f = torch.empty(self.R, **f64)
        u = torch.empty(self.N, **f64)
        torch.cuda.synchronize(self.dev)
        _check(lib().nmr_element_forces(self.h, _ptr(rt), _ptr(F), _ptr(f), _ptr(u)))
        return F, f, u


class Pool:
    """Fixed-capacity slot pool stepped by one captured graph (served form)."""

    def __init__(self, ctx: Context, capacity: int):
        h = C.c_void_p()
        _check(lib().nmr_pool_create(ctx.h, capacity, C.byref(h)))
        self.h, self.ctx, self.capacity = h, ctx, capacity

    def attach(self, inst: Instance) -> int:
        s = C.c_int()
        _check(lib().nmr_pool_attach(self.h, inst.h, C.byref(s)))
        return s.value

    def detach(self, slot: int):
        _check(lib().nmr_pool_detach(self.h, slot))

    def step(self, n_iters: int, status: bool = False, timing: bool = True):
        st = (C.c_int * self.capacity)() if status else None
        ms = C.c_float() if timing else None
        _check(lib().nmr_pool_step(self.h, n_iters, st, C.byref(ms) if timing else None))
        return (list(st) if status else None), (ms.value if timing else None)

    def close(self):
        if self.h:
            _check(lib().nmr_pool_destroy(self.h))
            self.h = None


class Coupled:
    """A core instance and rod instances tied to it (nmr_coupled_*); ties[k]
    is an (n_tie, 2) array of (rod vertex, core vertex) pairs of rod k."""

    def __init__(self, ctx: Context, core: Instance, rods: Sequence[Instance], ties, kappa: float):
        t = np.ascontiguousarray(np.stack([np.asarray(x) for x in ties]), dtype=np.int32)
        arr = (C.c_void_p * len(rods))(*[r.h.value for r in rods])
        h = C.c_void_p()
        _check(lib().nmr_coupled_create(ctx.h, core.h, len(rods), arr, t.ctypes.data_as(C.POINTER(C.c_int32)),
                                        t.shape[1], float(kappa), C.byref(h)))
        self.h = h
        self.n = 1 + len(rods)
        self.members = [core] + list(rods)

    def step(self, n_steps: int, n_iters: int, timings: bool = False):
        """Returns (status per member, core first; device ms per step or None)."""
        st = (C.c_int * self.n)()
        ms = (C.c_float * max(n_steps, 1))() if timings else None
        _check(lib().nmr_coupled_step(self.h, n_steps, n_iters, st, ms))
        return list(st), (list(ms)[:n_steps] if timings else None)

    def close(self):
        if self.h:
            _check(lib().nmr_coupled_destroy(self.h))
            self.h = None


class Trainer:
    """Neural cubature training (nmr_trainer_*) on an instance's mesh and
    decoder; `run` returns the loss histories and the elements added."""

    def __init__(self, inst: Instance, poses, wnet_weights, wnet_biases, wnet_scale: float, snet, n_c0: int, K: int,
                 epochs: int, c0=None, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, pose_chunk: int = 0):
        self.poses = np.ascontiguousarray(poses, np.float64)
        self.P, self.R = self.poses.shape
        self.m = int(inst.prob.tets.shape[0])
        self.N = inst.N
        self.K, self.epochs = K, epochs
        self.mlp = _Mlp(wnet_weights, wnet_biases, "identity")
        self.c_max = int(self.mlp.W[-1].shape[0])
        self.snet = np.ascontiguousarray(snet, np.float64)
        assert self.snet.size == 170
        self.c0 = None if c0 is None else np.ascontiguousarray(c0, np.int32)
        d = TrainDesc()
        d.n_poses, d.poses, d.c_max, d.n_c0 = self.P, self.poses.ctypes.data_as(_dp), self.c_max, n_c0
        d.c0 = None if self.c0 is None else self.c0.ctypes.data_as(C.POINTER(C.c_int32))
        d.K, d.epochs, d.lr, d.beta1, d.beta2, d.eps = K, epochs, lr, beta1, beta2, eps
        d.wnet, d.wnet_scale, d.snet = C.pointer(self.mlp.desc), wnet_scale, self.snet.ctypes.data_as(_dp)
        d.pose_chunk = pose_chunk
        h = C.c_void_p()
        _check(lib().nmr_trainer_create(inst.h, C.byref(d), C.byref(h)))
        self.h = h
        self.shapes = [W.shape for W in self.mlp.W]

    def run(self, n_alternations: int):
        """Returns (loss_w, loss_s [n_alt, epochs], added [n_alt, K], device ms)."""
        E, K = self.epochs, self.K
        lw = np.zeros((max(n_alternations, 1), E))
        ls = np.zeros((max(n_alternations, 1), E))
        add = np.zeros((max(n_alternations, 1), K), np.int32)
        ms = C.c_float()
        _check(lib().nmr_trainer_run(self.h, n_alternations, lw.ctypes.data_as(_dp), ls.ctypes.data_as(_dp),
                                     add.ctypes.data_as(C.POINTER(C.c_int)), C.byref(ms)))
        return lw[:n_alternations], ls[:n_alternations], add[:n_alternations], ms.value

    def get(self):
        """(C, weight-net Ws, bs, selection-net parameters)."""
        n = C.c_int()
        Cs = np.zeros(self.c_max, np.int32)
        nw = sum(a * b + a for a, b in self.shapes)
        wx = np.zeros(nw)
        th = np.zeros(170)
        _check(lib().nmr_trainer_get(self.h, C.byref(n), Cs.ctypes.data_as(C.POINTER(C.c_int32)),
                                     wx.ctypes.data_as(_dp), th.ctypes.data_as(_dp)))
        Ws, bs, o = [], [], 0
        for a, b in self.shapes:
            Ws.append(wx[o:o + a * b].reshape(a, b))
            o += a * b
            bs.append(wx[o:o + a].copy())
            o += a
        return Cs[:n.value].tolist(), Ws, bs, th

    def pose(self, p: int):
        """(F [n_tets, R], f [R], u [N]) of training pose p."""
        F = np.zeros((self.m, self.R))
        f = np.zeros(self.R)
        u = np.zeros(self.N)
        _check(lib().nmr_trainer_pose(self.h, p, F.ctypes.data_as(_dp), f.ctypes.data_as(_dp), u.ctypes.data_as(_dp)))
        return F, f, u

    def time_phase(self, phase: str, reps: int = 5) -> float:
        """Mean device microseconds of one phase (TRAIN_PHASES)."""
        us = C.c_float()
        _check(lib().nmr_trainer_time_phase(self.h, TRAIN_PHASES.index(phase), reps, C.byref(us)))
        return us.value

    def close(self):
        if self.h:
            _check(lib().nmr_trainer_destroy(self.h))
            self.h = None


def step_many(ctx: Context, insts: Sequence[Instance], n_steps: int, n_iters: int, timings: bool = True):
    """Advance all instances together; returns (status per instance, ms per step)."""
    n = len(insts)
    hs = (C.c_void_p * n)(*[x.h.value for x in insts])
    st = (C.c_int * n)()
    ms = (C.c_float * max(n_steps, 1))() if timings else None
    _check(lib().step_many(ctx.h, hs, n, n_steps, n_iters, st, ms))
    return list(st), (list(ms)[:n_steps] if timings else None)
