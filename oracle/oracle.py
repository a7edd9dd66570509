"""ctypes front end of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tdpd_oracle.c")
LIB = os.path.join(HERE, "libtdpd_oracle.so")

MAXT, MAXS = 4, 16
TERM = dict(cons=1, diss=2, rand=4, fick=8, frand=16, bond=32, bvisc=64, brand=128,
            area=256, vol=512, bend=1024, body=2048)
TERMS_ALL = sum(TERM.values())
FROZEN = 1 << 8


def build_oracle(force=True):
    """Compile the oracle with gcc (FP contraction off for the FP32 pair
    predicate, OpenMP for the CPU-baseline timing)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
               "-std=c11", "-D_GNU_SOURCE", SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [
        ("box", C.c_float * 3), ("rc", C.c_float), ("rcc", C.c_float),
        ("dt", C.c_double), ("kT", C.c_double), ("rho", C.c_double), ("m_s", C.c_double),
        ("s_exp", C.c_double), ("sc_exp", C.c_double),
        ("n_types", C.c_int32), ("n_species", C.c_int32),
        ("alpha", C.c_double * (MAXT * MAXT)), ("gamma", C.c_double * (MAXT * MAXT)),
        ("sigma", C.c_double * (MAXT * MAXT)), ("kappa", C.c_double * (MAXS * MAXT * MAXT)),
        ("body_force", C.c_double * 3), ("wall_axis", C.c_int32), ("wall_w", C.c_double),
        ("seed_lo", C.c_uint32), ("seed_hi", C.c_uint32), ("box_id", C.c_uint32),
        ("terms", C.c_int32), ("shear_rate", C.c_float),
        ("source", C.c_double * (MAXS * MAXT)), ("decay", C.c_double * (MAXS * MAXT)),
        ("wall_radius", C.c_double),
    ]


class _MeshParams(C.Structure):
    _fields_ = [(f, C.c_double) for f in
                ("p", "x0", "m_pow", "kb", "theta0", "kg", "kl", "kv", "gamma_t", "gamma_c")]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(_Params)]
        L.orc_set_params.argtypes = [P, C.POINTER(_Params)]
        L.orc_destroy.argtypes = [P]
        L.orc_add_mesh.restype = C.c_int
        L.orc_add_mesh.argtypes = [P, C.c_int, C.c_int, P, P, C.POINTER(_MeshParams)]
        L.orc_add_rbc.restype = C.c_int
        L.orc_add_rbc.argtypes = [P, C.c_int, C.c_int64]
        L.orc_mesh_info.argtypes = [P, C.c_int, P]
        L.orc_mesh_topology.argtypes = [P, C.c_int, P, P]
        L.orc_pairs.argtypes = [P, C.c_int64, P, C.c_int, C.c_int, C.c_uint32, C.c_int64, P, P,
                                P]
        L.orc_forces.restype = C.c_int
        L.orc_forces.argtypes = [P, C.c_int64, P, P, P, P, C.c_uint32, P, P, P, P, P, P, P, P, P]
        L.orc_membrane.restype = C.c_int
        L.orc_membrane.argtypes = [P, C.c_int64, P, P, C.c_uint32, P, P, P]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [P, C.c_int64, P, P, P, P, P, P, C.c_uint32, P]
        L.orc_diag.argtypes = [P, C.c_int64, P, P, P, P]
        L.orc_philox4x32.argtypes = [P, P, C.c_int, P]
        L.orc_pair_normals_batch.argtypes = [C.POINTER(_Params), C.c_uint32, C.c_int64, P, P,
                                             C.c_uint32, P]
        L.orc_pair_normals4.argtypes = [C.POINTER(_Params), C.c_uint32, C.c_uint32,
                                        C.c_uint32, C.c_uint32, P]
        L.orc_disp.restype = C.c_float
        L.orc_disp.argtypes = [P, P, P, C.c_uint32, P]
        L.orc_u01.restype = C.c_double
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_pair_normals.argtypes = [C.POINTER(_Params), C.c_uint32, C.c_uint32,
                                       C.c_uint32, C.c_uint32, P]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def philox4x32(ctr, key, rounds=10):
    L = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    L.orc_philox4x32(_ptr(c), _ptr(k), rounds, _ptr(out))
    return out


def u01(bits):
    return _load().orc_u01(int(bits))


def _params_from(cfg, terms=TERMS_ALL):
    p = _Params()
    for a in range(3):
        p.box[a] = cfg.box[a]
    p.rc, p.rcc = cfg.rc, cfg.rcc
    p.dt, p.kT, p.rho, p.m_s = cfg.dt, cfg.kT, cfg.rho, cfg.m_s
    p.s_exp, p.sc_exp = cfg.s_exp, cfg.sc_exp
    T, S = cfg.n_types, cfg.n_species
    assert T <= MAXT and S <= MAXS
    p.n_types, p.n_species = T, S
    for i in range(T):
        for j in range(T):
            p.alpha[i * T + j] = cfg.alpha[i, j]
            p.gamma[i * T + j] = cfg.gamma[i, j]
            p.sigma[i * T + j] = cfg.sigma[i, j]
            for s in range(S):
                p.kappa[(s * T + i) * T + j] = cfg.kappa[s, i, j]
    for a in range(3):
        p.body_force[a] = cfg.body_force[a]
    p.wall_axis, p.wall_w = cfg.wall_axis, cfg.wall_w
    p.seed_lo = cfg.seed & 0xFFFFFFFF
    p.seed_hi = (cfg.seed >> 32) & 0xFFFFFFFF
    p.box_id = cfg.box_id
    p.terms = terms
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


def pair_normals(cfg, k, gi, gj, stream):
    p = _params_from(cfg)
    out = np.zeros(2)
    _load().orc_pair_normals(C.byref(p), k, gi, gj, stream, _ptr(out))
    return out


def pair_normals4(cfg, k, gi, gj, stream):
    p = _params_from(cfg)
    out = np.zeros(4)
    _load().orc_pair_normals4(C.byref(p), k, gi, gj, stream, _ptr(out))
    return out


def pair_normals_batch(cfg, k, gi, gj, stream=0):
    p = _params_from(cfg)
    gi = np.ascontiguousarray(gi, dtype=np.uint32)
    gj = np.ascontiguousarray(gj, dtype=np.uint32)
    out = np.zeros((gi.shape[0], 2))
    _load().orc_pair_normals_batch(C.byref(p), k, gi.shape[0], _ptr(gi), _ptr(gj), stream,
                                   _ptr(out))
    return out


class Oracle:
    """FP64 oracle bound to one configuration (an inputs.Config)."""

    def __init__(self, cfg, terms=TERMS_ALL):
        self.cfg = cfg
        self.L = _load()
        self.terms = terms
        self._p = _params_from(cfg, terms)
        self.h = self.L.orc_create(C.byref(self._p))
        self.mesh_ids = []
        if cfg.mesh_xyz is not None:
            mp = cfg.mesh_params
            m = _MeshParams(p=mp.p, x0=mp.x0, m_pow=mp.m_pow, kb=mp.kb, theta0=mp.theta0,
                            kg=mp.kg, kl=mp.kl, kv=mp.kv, gamma_t=mp.gamma_t,
                            gamma_c=mp.gamma_c)
            tri = np.ascontiguousarray(cfg.mesh_tri, dtype=np.int32)
            ref = np.ascontiguousarray(cfg.mesh_xyz, dtype=np.float64)
            mid = self.L.orc_add_mesh(self.h, ref.shape[0], tri.shape[0], _ptr(tri),
                                      _ptr(ref), C.byref(m))
            if mid < 0:
                raise ValueError(f"oracle rejected mesh ({mid})")
            self.mesh_ids.append(mid)
            for g0 in cfg.rbc_first_gid:
                self.L.orc_add_rbc(self.h, mid, int(g0))
        self.n_rbc = len(cfg.rbc_first_gid) if cfg.mesh_xyz is not None else 0

    def __del__(self):
        try:
            self.L.orc_destroy(self.h)
        except Exception:
            pass

    def set_terms(self, terms):
        self.terms = terms
        self._p.terms = terms
        self.L.orc_set_params(self.h, C.byref(self._p))

    def mesh_info(self, mesh=0):
        out = np.zeros(6)
        self.L.orc_mesh_info(self.h, mesh, _ptr(out))
        return dict(A0=out[0], V0=out[1], theta0=out[2], nedge=int(out[3]),
                    ndih=int(out[4]), ntri=int(out[5]))

    def mesh_topology(self, mesh=0):
        info = self.mesh_info(mesh)
        e = np.zeros((info["nedge"], 2), dtype=np.int32)
        d = np.zeros((info["ndih"], 4), dtype=np.int32)
        self.L.orc_mesh_topology(self.h, mesh, _ptr(e), _ptr(d))
        return e, d

    def disp(self, xi, xj, k=0):
        a = np.ascontiguousarray(xi, dtype=np.float32)
        b = np.ascontiguousarray(xj, dtype=np.float32)
        d = np.zeros(3, dtype=np.float32)
        d2 = self.L.orc_disp(self.h, _ptr(a), _ptr(b), int(k), _ptr(d))
        return d, np.float32(d2)

    def pairs(self, pos_f32, which=0, brute=False, cap=None, k=0):
        x = np.ascontiguousarray(pos_f32, dtype=np.float32)
        n = x.shape[0]
        if cap is None:
            cap = max(16, n * 80)
        out = np.zeros((cap, 2), dtype=np.int32)
        cnt = np.zeros(1, dtype=np.int64)
        nz = np.zeros(1, dtype=np.int64)
        self.L.orc_pairs(self.h, n, _ptr(x), which, int(brute), int(k), cap, _ptr(out),
                         _ptr(cnt), _ptr(nz))
        m = int(cnt[0])
        if m > cap:
            return self.pairs(x, which, brute, cap=m, k=k)
        return out[:m].copy(), int(nz[0])

    def forces(self, pos, vel, conc, flags=None, k=0, which=None, energy=False):
        cfg = self.cfg
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        conc = np.ascontiguousarray(conc, dtype=np.float64).reshape(pos.shape[0], cfg.n_species)
        n = pos.shape[0]
        flags = np.ascontiguousarray(cfg.flags if flags is None else flags, dtype=np.uint32)
        F = np.zeros((n, 3))
        Q = np.zeros((n, cfg.n_species))
        av = np.zeros((max(self.n_rbc, 1), 2))
        en = np.zeros(4)
        nz = np.zeros(1, dtype=np.int64)
        w = None if which is None else np.ascontiguousarray(which, dtype=np.uint8)
        Fa = np.zeros(n)
        Fm = np.zeros(n)
        Qa = np.zeros((n, cfg.n_species))
        err = self.L.orc_forces(self.h, n, _ptr(pos), _ptr(vel), _ptr(conc), _ptr(flags), k,
                                _ptr(w), _ptr(F), _ptr(Q), _ptr(av), _ptr(en), _ptr(nz), _ptr(Fa),
                                _ptr(Qa), _ptr(Fm))
        # Fabs/Qabs: sum over contributions of their magnitudes (the scale of
        # the rounding error of an FP32 sum of the same terms); Fmabs: the
        # membrane terms' share of Fabs
        res = dict(F=F, Q=Q, av=av[:self.n_rbc], err=err, nzero=int(nz[0]), Fabs=Fa, Qabs=Qa,
                   Fmabs=Fm)
        if energy:
            res["energy"] = en
        return res

    def membrane(self, pos, vel=None, k=0):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        n = pos.shape[0]
        vel = np.zeros_like(pos) if vel is None else np.ascontiguousarray(vel, dtype=np.float64)
        F = np.zeros((n, 3))
        en = np.zeros(4)
        av = np.zeros((max(self.n_rbc, 1), 2))
        err = self.L.orc_membrane(self.h, n, _ptr(pos), _ptr(vel), k, _ptr(F), _ptr(en),
                                  _ptr(av))
        return dict(F=F, energy=en, av=av[:self.n_rbc], err=err)

    def step(self, state, k):
        """One velocity-Verlet step in place on a dict of float64 arrays
        pos, vel, conc, F, Q (flags from the config)."""
        flags = np.ascontiguousarray(self.cfg.flags, dtype=np.uint32)
        av = np.zeros((max(self.n_rbc, 1), 2))
        n = state["pos"].shape[0]
        err = self.L.orc_step(self.h, n, _ptr(state["pos"]), _ptr(state["vel"]),
                              _ptr(state["conc"]), _ptr(state["F"]), _ptr(state["Q"]),
                              _ptr(flags), k, _ptr(av))
        state["av"] = av[:self.n_rbc]
        return err

    def init_state(self, k=0):
        cfg = self.cfg
        st = dict(pos=cfg.pos.astype(np.float64), vel=cfg.vel.astype(np.float64),
                  conc=cfg.conc.astype(np.float64))
        r = self.forces(st["pos"], st["vel"], st["conc"], k=k)
        st["F"], st["Q"] = r["F"], r["Q"]
        return st

    def diag(self, vel, conc, flags=None):
        cfg = self.cfg
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        conc = np.ascontiguousarray(conc, dtype=np.float64)
        flags = np.ascontiguousarray(cfg.flags if flags is None else flags, dtype=np.uint32)
        out = np.zeros(4 + cfg.n_species)
        self.L.orc_diag(self.h, vel.shape[0], _ptr(vel), _ptr(conc), _ptr(flags), _ptr(out))
        return dict(P=out[:3], kT=out[3], C=out[4:])
