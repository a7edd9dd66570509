"""Python binding of libtdpd.so (include/tdpd.h): argument marshalling only.

Every function below forwards to the C entry point of the same name; all
computation runs in the library's HIP kernels.  Device memory comes from
torch's caching allocator through the library's allocator callback, and
kernels are enqueued on torch's current HIP stream.  The library must have
been built (paper_1611_06163_amd/build.py); importing this module on a
machine where it is missing raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdpd.so")

MAX_TYPES, MAX_SPECIES = 4, 16
TERM = dict(cons=1, diss=2, rand=4, fick=8, frand=16, bond=32, bvisc=64, brand=128,
            area=256, vol=512, bend=1024, body=2048)
TERMS_ALL = 4095
FLAG_FROZEN = 1 << 8
PHASE = dict(pair=1, bin=2, membrane=4, kick=8)
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "BOX_TOO_SMALL", -3: "OOM", -4: "HIP",
          -5: "NONFINITE", -6: "BOND_OVEREXTENDED", -7: "STATE", -8: "UNSUPPORTED",
          -9: "CAPACITY", -10: "IO", -11: "LIST"}


class TdpdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class tdpd_params(C.Structure):
    _fields_ = [
        ("box", C.c_float * 3), ("rc", C.c_float), ("rcc", C.c_float), ("dt", C.c_float),
        ("kT", C.c_float), ("rho", C.c_float), ("m_s", C.c_float), ("s_exp", C.c_float),
        ("sc_exp", C.c_float), ("n_types", C.c_int32), ("n_species", C.c_int32),
        ("alpha", C.c_float * (MAX_TYPES * MAX_TYPES)),
        ("gamma", C.c_float * (MAX_TYPES * MAX_TYPES)),
        ("sigma", C.c_float * (MAX_TYPES * MAX_TYPES)),
        ("kappa", C.c_float * (MAX_SPECIES * MAX_TYPES * MAX_TYPES)),
        ("body_force", C.c_float * 3), ("wall_axis", C.c_int32), ("wall_w", C.c_float),
        ("seed", C.c_uint64), ("box_id", C.c_uint32), ("terms", C.c_int32),
        ("shear_rate", C.c_float),
        ("source", C.c_float * (MAX_SPECIES * MAX_TYPES)),
        ("decay", C.c_float * (MAX_SPECIES * MAX_TYPES)),
        ("wall_radius", C.c_float),
    ]


class tdpd_box(C.Structure):
    _fields_ = [("box", C.c_float * 3), ("seed", C.c_uint64), ("box_id", C.c_uint32),
                ("shear_rate", C.c_float)]


class tdpd_mesh_params(C.Structure):
    _fields_ = [(f, C.c_float) for f in
                ("p", "x0", "m_pow", "kb", "theta0", "kg", "kl", "kv", "gamma_t", "gamma_c")]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None


def lib():
    """Load libtdpd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1611_06163_amd.build` (hipcc, gfx950)")
        # torch's HIP runtime must be the process's only one: load it before
        # libtdpd.so so that the library's libamdhip64 dependency binds to it
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "tdpd_create": (C.c_int, [C.POINTER(tdpd_params), P, ALLOC_FN, FREE_FN, P,
                                      C.POINTER(P)]),
            "tdpd_create_batch": (C.c_int, [C.POINTER(tdpd_params), I32, P, P, ALLOC_FN,
                                            FREE_FN, P, C.POINTER(P)]),
            "tdpd_set_state": (C.c_int, [P, I64, P, P, P, P]),
            "tdpd_set_state_boxes": (C.c_int, [P, P, P, P, P, P]),
            "tdpd_num_boxes": (I32, [P]),
            "tdpd_add_mesh": (C.c_int, [P, I32, P, I32, P, C.POINTER(tdpd_mesh_params),
                                        C.POINTER(I32)]),
            "tdpd_add_rbc": (C.c_int, [P, I32, I64, C.POINTER(I32)]),
            "tdpd_compute_forces": (C.c_int, [P, C.c_uint32]),
            "tdpd_step": (C.c_int, [P, I32]),
            "tdpd_sync": (C.c_int, [P]),
            "tdpd_get_state": (C.c_int, [P, P, P, P]),
            "tdpd_get_forces": (C.c_int, [P, P, P]),
            "tdpd_get_pairs": (C.c_int, [P, I32, I64, P, C.POINTER(I64)]),
            "tdpd_diagnostics": (C.c_int, [P, P, I64]),
            "tdpd_diagnostics_noalloc": (C.c_int, [P, P, I64]),
            "tdpd_set_timing": (C.c_int, [P, I32]),
            "tdpd_get_timing": (C.c_int, [P, I32, C.POINTER(C.c_double), C.POINTER(I64)]),
            "tdpd_autotune": (C.c_int, [P, C.c_char_p, I32, C.POINTER(C.c_double)]),
            "tdpd_set_tile": (C.c_int, [P, I32, I32, I32, I32]),
            "tdpd_set_verlet": (C.c_int, [P, C.c_float, I32, I32]),
            "tdpd_get_verlet": (C.c_int, [P, C.POINTER(C.c_float), C.POINTER(I32), C.POINTER(I32)]),
            "tdpd_get_tile": (C.c_int, [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32),
                                        C.POINTER(I32)]),
            "tdpd_mlp_create": (C.c_int, [P, ALLOC_FN, FREE_FN, P, C.POINTER(P)]),
            "tdpd_mlp_num_params": (I64, []),
            "tdpd_mlp_set_params": (C.c_int, [P, P]),
            "tdpd_mlp_get_params": (C.c_int, [P, P]),
            "tdpd_mlp_forward": (C.c_int, [P, P, I64, P]),
            "tdpd_mlp_forward_hidden": (C.c_int, [P, P, I64, P, P]),
            "tdpd_mlp_loss_grad": (C.c_int, [P, P, P, I64, C.c_float, C.POINTER(C.c_double), P]),
            "tdpd_mlp_train": (C.c_int, [P, P, P, I64, C.c_float, I32, I32, C.c_float, P]),
            "tdpd_mlp_last_error": (C.c_char_p, [P]),
            "tdpd_mlp_destroy": (None, [P]),
            "tdpd_surrogate_sample": (C.c_int, [P, P, P, P]),
            "tdpd_surrogate_enable": (C.c_int, [P, P, C.c_float, C.c_float, I32]),
            "tdpd_surrogate_disable": (C.c_int, [P]),
            "tdpd_surrogate_stats": (C.c_int, [P, P]),
            "tdpd_save": (C.c_int, [P, C.c_char_p]),
            "tdpd_load": (C.c_int, [P, C.c_char_p]),
            "tdpd_num_particles": (I64, [P]),
            "tdpd_step_counter": (I64, [P]),
            "tdpd_coincident_pairs": (I64, [P]),
            "tdpd_last_error": (C.c_char_p, [P]),
            "tdpd_destroy": (None, [P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return [n for n in dir(lib()) if n.startswith("tdpd_")]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def params_from_config(cfg, terms=TERMS_ALL):
    p = tdpd_params()
    for a in range(3):
        p.box[a] = cfg.box[a]
        p.body_force[a] = cfg.body_force[a]
    p.rc, p.rcc, p.dt, p.kT, p.rho, p.m_s = cfg.rc, cfg.rcc, cfg.dt, cfg.kT, cfg.rho, cfg.m_s
    p.s_exp, p.sc_exp = cfg.s_exp, cfg.sc_exp
    T, S = cfg.n_types, cfg.n_species
    p.n_types, p.n_species = T, S
    for i in range(T):
        for j in range(T):
            p.alpha[i * T + j] = cfg.alpha[i, j]
            p.gamma[i * T + j] = cfg.gamma[i, j]
            p.sigma[i * T + j] = cfg.sigma[i, j]
            for s in range(S):
                p.kappa[(s * T + i) * T + j] = cfg.kappa[s, i, j]
    p.wall_axis, p.wall_w = cfg.wall_axis, cfg.wall_w
    p.seed, p.box_id, p.terms = cfg.seed, cfg.box_id, terms
    p.shear_rate = float(getattr(cfg, "shear_rate", 0.0))
    for name in ("source", "decay"):
        a = getattr(cfg, name, None)
        if a is not None:
            a = np.asarray(a, dtype=np.float64).reshape(S, T)
            for s in range(S):
                for t in range(T):
                    getattr(p, name)[s * T + t] = a[s, t]
    p.wall_radius = float(getattr(cfg, "wall_radius", 0.0))
    return p


class _TorchAllocator:
    """Allocator callback backed by torch's caching allocator."""

    def __init__(self, device=0):
        import torch
        self.torch = torch
        self.device = device
        self.live = {}
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=f"cuda:{self.device}")
        except Exception:
            return None
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, user):
        self.live.pop(ptr, None)


class System:
    """One tDPD system on the GPU (a thin owner of a tdpd_sys handle).

    `cfg` is one inputs.Config (one periodic box) or a list of them (a
    batched ensemble: one box per config, sharing the common parameters of
    the first; particles concatenated box-major)."""

    def __init__(self, cfg, terms=TERMS_ALL, stream=None, torch_alloc=True):
        L = lib()
        cfgs = list(cfg) if isinstance(cfg, (list, tuple)) else [cfg]
        self.cfgs = cfgs
        self.cfg = cfgs[0]
        self.S = self.cfg.n_species
        self._alloc = None
        alloc_cb, free_cb = ALLOC_FN(), FREE_FN()
        if torch_alloc:
            self._alloc = _TorchAllocator()
            alloc_cb, free_cb = self._alloc.alloc_cb, self._alloc.free_cb
        if stream is None and torch_alloc:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        self._p = params_from_config(self.cfg, terms)
        h = C.c_void_p()
        strm = C.c_void_p(stream) if stream else None
        batched = isinstance(cfg, (list, tuple))
        if batched:
            boxes = (tdpd_box * len(cfgs))()
            for b, c in enumerate(cfgs):
                for a in range(3):
                    boxes[b].box[a] = c.box[a]
                boxes[b].seed, boxes[b].box_id = c.seed, c.box_id
                boxes[b].shear_rate = getattr(c, "shear_rate", 0.0)
            rc = L.tdpd_create_batch(C.byref(self._p), len(cfgs), C.cast(boxes, C.c_void_p), strm,
                                     alloc_cb, free_cb, None, C.byref(h))
        else:
            rc = L.tdpd_create(C.byref(self._p), strm, alloc_cb, free_cb, None, C.byref(h))
        if rc:
            raise TdpdError(rc, "tdpd_create rejected the parameters")
        self.h = h
        counts = np.array([c.n for c in cfgs], dtype=np.int64)
        self.box_offset = np.concatenate([[0], np.cumsum(counts)])
        cat = lambda f, dt: np.ascontiguousarray(
            np.concatenate([getattr(c, f) for c in cfgs]) if cfgs else np.zeros(0), dt)
        self._check(L.tdpd_set_state_boxes(self.h, _ptr(counts), _ptr(cat("pos", np.float32)),
                                           _ptr(cat("vel", np.float32)),
                                           _ptr(cat("conc", np.float32)),
                                           _ptr(cat("flags", np.uint32))))
        self.n = int(counts.sum())
        self.rbc_first = []
        mesh_cfg = next((c for c in cfgs if c.mesh_xyz is not None and len(c.rbc_first_gid)), None)
        if mesh_cfg is not None:
            mp = mesh_cfg.mesh_params
            m = tdpd_mesh_params(p=mp.p, x0=mp.x0, m_pow=mp.m_pow, kb=mp.kb,
                                 theta0=mp.theta0, kg=mp.kg, kl=mp.kl, kv=mp.kv,
                                 gamma_t=mp.gamma_t, gamma_c=mp.gamma_c)
            ref = np.ascontiguousarray(mesh_cfg.mesh_xyz, np.float64)
            tri = np.ascontiguousarray(mesh_cfg.mesh_tri, np.int32)
            mid = C.c_int32()
            self._check(L.tdpd_add_mesh(self.h, ref.shape[0], _ptr(ref), tri.shape[0], _ptr(tri),
                                        C.byref(m), C.byref(mid)))
            for b, c in enumerate(cfgs):
                if not len(c.rbc_first_gid):
                    continue
                if c.mesh_xyz is not mesh_cfg.mesh_xyz and not (
                        np.array_equal(c.mesh_xyz, mesh_cfg.mesh_xyz)
                        and np.array_equal(c.mesh_tri, mesh_cfg.mesh_tri)):
                    raise ValueError("all boxes of a batch must share one cell mesh")
                for g0 in c.rbc_first_gid:
                    rid = C.c_int32()
                    g = int(self.box_offset[b] + g0)
                    self._check(L.tdpd_add_rbc(self.h, mid.value, g, C.byref(rid)))
                    self.rbc_first.append(g)

    def _check(self, rc):
        if rc:
            msg = lib().tdpd_last_error(self.h).decode() if getattr(self, "h", None) else ""
            raise TdpdError(rc, msg)

    def close(self):
        if getattr(self, "h", None):
            lib().tdpd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        self._check(lib().tdpd_step(self.h, int(n)))

    def compute_forces(self, k=0):
        self._check(lib().tdpd_compute_forces(self.h, int(k)))

    def sync(self):
        self._check(lib().tdpd_sync(self.h))

    def get_state(self):
        pos = np.empty((self.n, 3), np.float32)
        vel = np.empty((self.n, 3), np.float32)
        conc = np.empty((self.n, self.S), np.float32)
        self._check(lib().tdpd_get_state(self.h, _ptr(pos), _ptr(vel), _ptr(conc)))
        return pos, vel, conc

    def get_forces(self):
        F = np.empty((self.n, 3), np.float32)
        Q = np.empty((self.n, self.S), np.float32)
        self._check(lib().tdpd_get_forces(self.h, _ptr(F), _ptr(Q)))
        return F, Q

    def pairs(self, which=0, cap=None):
        cap = max(16, self.n * 80) if cap is None else cap
        out = np.empty((cap, 2), np.int32)
        cnt = C.c_int64()
        rc = lib().tdpd_get_pairs(self.h, which, cap, _ptr(out), C.byref(cnt))
        if rc == -9:
            return self.pairs(which, cap=int(cnt.value))
        self._check(rc)
        return out[:cnt.value].copy()

    def diagnostics(self):
        nrbc = len(self.rbc_first)
        out = np.zeros(4 + self.S + 2 * nrbc)
        self._check(lib().tdpd_diagnostics(self.h, _ptr(out), out.size))
        return dict(P=out[:3], kT=out[3], C=out[4:4 + self.S],
                    av=out[4 + self.S:].reshape(nrbc, 2))

    def diagnostics_noalloc(self, out_dev_ptr, cap):
        """Enqueue the diagnostics into a caller-owned device buffer of `cap`
        doubles (address as an int) on the library's stream; no allocation,
        no wait."""
        self._check(lib().tdpd_diagnostics_noalloc(self.h, C.c_void_p(int(out_dev_ptr)),
                                                   int(cap)))

    def surrogate_sample(self):
        """Inputs X [nv][20], plain bending + local-area targets in the local
        frame T [nv][3] and the may-use mask of every membrane vertex."""
        nv = sum(len(c.rbc_first_gid) * c.mesh_xyz.shape[0] for c in self.cfgs
                 if c.mesh_xyz is not None)
        X = np.empty((nv, 20), np.float32)
        T = np.empty((nv, 3), np.float32)
        ok = np.empty(nv, np.uint8)
        self._check(lib().tdpd_surrogate_sample(self.h, _ptr(X), _ptr(T), _ptr(ok)))
        return X, T, ok.astype(bool)

    def surrogate_enable(self, mlp, force_scale, tol=1e-2, check_every=10):
        self._check(lib().tdpd_surrogate_enable(self.h, mlp.h, float(force_scale), float(tol),
                                                int(check_every)))

    def surrogate_disable(self):
        self._check(lib().tdpd_surrogate_disable(self.h))

    def surrogate_stats(self):
        out = np.zeros(4)
        self._check(lib().tdpd_surrogate_stats(self.h, _ptr(out)))
        return dict(on_network=out[0], max_err=out[1], mean_err=out[2], eligible=out[3])

    def autotune(self, cache_path=None, reps=5):
        """Pick the fastest tile shape of the pair kernel (returns its ms)."""
        ms = C.c_double()
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(lib().tdpd_autotune(self.h, path, int(reps), C.byref(ms)))
        return ms.value

    @property
    def tile(self):
        """(waves, chunks, split, filter) of the cell-tiled pair kernel."""
        w, c, sp, f = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        self._check(lib().tdpd_get_tile(self.h, C.byref(w), C.byref(c), C.byref(sp), C.byref(f)))
        return (w.value, c.value, sp.value, f.value)

    @tile.setter
    def tile(self, t):
        self._check(lib().tdpd_set_tile(self.h, int(t[0]), int(t[1]), int(t[2]), int(t[3])))

    def set_verlet(self, skin, every, capacity=0):
        """Neighbour lists of radius max(rc, rcc) + skin, rebuilt every `every` steps."""
        self._check(lib().tdpd_set_verlet(self.h, float(skin), int(every), int(capacity)))

    @property
    def verlet(self):
        """(skin, every, capacity) of the neighbour lists; every 0: per-step cells."""
        sk, ev, cap = C.c_float(), C.c_int32(), C.c_int32()
        self._check(lib().tdpd_get_verlet(self.h, C.byref(sk), C.byref(ev), C.byref(cap)))
        return (sk.value, ev.value, cap.value)

    def save(self, path):
        self._check(lib().tdpd_save(self.h, os.fsencode(path)))

    def load(self, path):
        self._check(lib().tdpd_load(self.h, os.fsencode(path)))

    def set_timing(self, mask):
        self._check(lib().tdpd_set_timing(self.h, int(mask)))

    def get_timing(self, phase):
        ms, cnt = C.c_double(), C.c_int64()
        self._check(lib().tdpd_get_timing(self.h, int(phase), C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    @property
    def step_counter(self):
        return int(lib().tdpd_step_counter(self.h))

    @property
    def coincident_pairs(self):
        return int(lib().tdpd_coincident_pairs(self.h))


class Mlp:
    """The membrane-surrogate network of libtdpd (tdpd_mlp_*): parameters and
    Adam moments on the device; forward pass, gradient and training run in
    the library's kernels."""

    def __init__(self, params=None, stream=None):
        L = lib()
        self._alloc = _TorchAllocator()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        rc = L.tdpd_mlp_create(C.c_void_p(stream) if stream else None, self._alloc.alloc_cb,
                               self._alloc.free_cb, None, C.byref(h))
        if rc:
            raise TdpdError(rc, "tdpd_mlp_create failed")
        self.h = h
        self.n_params = int(L.tdpd_mlp_num_params())
        if params is not None:
            self.set_params(params)

    def _check(self, rc):
        if rc:
            raise TdpdError(rc, lib().tdpd_mlp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().tdpd_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.n_params
        self._check(lib().tdpd_mlp_set_params(self.h, _ptr(p)))

    def get_params(self):
        p = np.empty(self.n_params, np.float32)
        self._check(lib().tdpd_mlp_get_params(self.h, _ptr(p)))
        return p

    def forward(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.empty((X.shape[0], 3), np.float32)
        self._check(lib().tdpd_mlp_forward(self.h, _ptr(X), X.shape[0], _ptr(Y)))
        return Y

    def forward_hidden(self, X):
        """Y [n][3] and the hidden layers' FP32 activations H [3][n][128]
        (before their bfloat16 rounding)."""
        X = np.ascontiguousarray(X, dtype=np.float32)
        n = X.shape[0]
        Y = np.empty((n, 3), np.float32)
        H = np.empty((3, n, 128), np.float32)
        self._check(lib().tdpd_mlp_forward_hidden(self.h, _ptr(X), n, _ptr(Y), _ptr(H)))
        return Y, H

    def loss_grad(self, X, T, target_scale=1.0):
        X = np.ascontiguousarray(X, dtype=np.float32)
        T = np.ascontiguousarray(T, dtype=np.float32)
        loss = C.c_double()
        g = np.empty(self.n_params, np.float32)
        self._check(lib().tdpd_mlp_loss_grad(self.h, _ptr(X), _ptr(T), X.shape[0],
                                             float(target_scale), C.byref(loss), _ptr(g)))
        return loss.value, g

    def train(self, X, T, target_scale, batch, steps, lr):
        X = np.ascontiguousarray(X, dtype=np.float32)
        T = np.ascontiguousarray(T, dtype=np.float32)
        losses = np.empty(max(int(steps), 1))
        self._check(lib().tdpd_mlp_train(self.h, _ptr(X), _ptr(T), X.shape[0],
                                         float(target_scale), int(batch), int(steps), float(lr),
                                         _ptr(losses)))
        return losses[:int(steps)]
