"""FP64 CPU oracle for CRBM-aided Monte Carlo (arXiv:2008.05401).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU leg of
the benchmark are the only callers.  The GPU product path never imports this
package and shares no code with it.

This module is a thin ctypes harness around ``crbm_oracle.c`` (plain C, FP64,
built with -O2 -ffp-contract=off, no fast-math).  Arrays are numpy; states are
+-1 int8 with layout [chain][C][L][L].
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "crbm_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

ISING, KITAEV, GIBBS = 0, 1, 2
ST_INIT, ST_HID, ST_VIS, ST_MH, ST_PT = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile the oracle library in-tree with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_SRC) > os.path.getmtime(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(ct.Structure):
    _fields_ = [("K", ct.c_int32), ("C", ct.c_int32), ("Lw", ct.c_int32),
                ("W", ct.c_void_p), ("hbias", ct.c_void_p), ("vbias", ct.c_void_p),
                ("open_cols", ct.c_int32), ("n_edge", ct.c_int32), ("dense", ct.c_int32)]


class _RunDesc(ct.Structure):
    _fields_ = [("target", ct.c_int32), ("L", ct.c_int32), ("n_chains", ct.c_int32),
                ("gibbs_k", ct.c_int32), ("burnin", ct.c_int32), ("g0", ct.c_uint32),
                ("seed", ct.c_uint64), ("J", ct.c_double * 3), ("boundary", ct.c_int32)]


CHAIN_DTYPE = np.dtype([
    ("sweeps", "<i8"), ("n_acc", "<i8"), ("n_meas", "<i8"), ("pad0", "<i8"),
    ("sumE", "<i8"), ("sumE2", "<i8"), ("sumM", "<i8"), ("sumAbsM", "<i8"), ("sumM2", "<i8"),
    ("E", "<i8"), ("F", "<f8"), ("S", "<f8"), ("Ef", "<f8"), ("Cf", "<f8"),
    ("kE", "<f8"), ("kE2", "<f8"), ("kCf", "<f8"), ("n_swap", "<i8"),
])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ct.CDLL(_LIB)
        P = ct.POINTER
        vp = ct.c_void_p
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_mh_uniform.argtypes = [ct.c_uint64, ct.c_uint32, ct.c_uint32]
        L.orc_mh_uniform.restype = ct.c_double
        L.orc_unit_uniform.argtypes = [ct.c_uint64, ct.c_uint32, ct.c_uint32, ct.c_uint32, ct.c_uint32]
        L.orc_unit_uniform.restype = ct.c_double
        L.orc_hidden_preact.argtypes = [P(_Params), vp, ct.c_int, vp]
        L.orc_visible_preact.argtypes = [P(_Params), vp, ct.c_int, vp]
        L.orc_free_energy.argtypes = [P(_Params), vp, ct.c_int, ct.c_int, vp]
        L.orc_ising_energy.argtypes = [vp, ct.c_int, ct.c_int]
        L.orc_ising_energy.restype = ct.c_int64
        L.orc_magnetization.argtypes = [vp, ct.c_int]
        L.orc_magnetization.restype = ct.c_int64
        L.orc_kitaev_matrix.argtypes = [vp, ct.c_int, ct.c_int, vp, ct.c_int, vp]
        L.orc_singular_values.argtypes = [vp, ct.c_int, vp]
        L.orc_singular_values.restype = ct.c_int
        L.orc_kitaev_S.argtypes = [vp, ct.c_int, ct.c_int, vp, ct.c_int, ct.c_double, vp, vp, vp]
        L.orc_kitaev_S.restype = ct.c_double
        L.orc_target.argtypes = [ct.c_int, vp, ct.c_int, ct.c_int, ct.c_int, ct.c_int, vp, vp, vp, vp]
        L.orc_init_state.argtypes = [ct.c_uint64, ct.c_uint32, ct.c_int, ct.c_int, ct.c_int, vp]
        L.orc_gibbs_step.argtypes = [P(_Params), ct.c_int, vp, vp, vp, ct.c_uint64, ct.c_uint32,
                                     ct.c_uint32, ct.c_uint32, vp]
        L.orc_gibbs_step.restype = ct.c_int64
        L.orc_chain_init.argtypes = [P(_Params), P(_RunDesc), vp, vp, vp, vp]
        L.orc_run.argtypes = [P(_Params), P(_RunDesc), vp, vp, vp, vp, ct.c_uint32, ct.c_int, vp, vp, vp, vp]
        L.orc_tempering_swap.argtypes = [P(_RunDesc), ct.c_int, vp, vp, vp, vp, ct.c_int, ct.c_uint32, vp]
        L.orc_pt_uniform.argtypes = [ct.c_uint64, ct.c_uint32, ct.c_uint32]
        L.orc_pt_uniform.restype = ct.c_double
        L.orc_grad.argtypes = [P(_Params), vp, ct.c_int, ct.c_int, vp, vp, vp, vp]
        L.orc_num_threads.restype = ct.c_int
        L.orc_set_threads.argtypes = [ct.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


class CRBM:
    """CRBM parameters as float32 numpy arrays: W[K][C][Lw][Lw], hbias[K], vbias[C].

    The locally connected CRBM of Sec. IV.B takes W[1+2n][K][C][Lw][Lw] and
    hbias[1+2n][K] (bank 0 the bulk, banks 1..n the left hidden columns
    0..n-1, banks n+1..2n the right columns L-n..L-1) with open_cols=True:
    filter windows do not wrap across the column edge."""

    def __init__(self, W, hbias, vbias, open_cols=None):
        self.W = np.ascontiguousarray(W, dtype=np.float32)
        assert self.W.ndim in (4, 5) and self.W.shape[-1] == self.W.shape[-2]
        self.banks = 1 if self.W.ndim == 4 else self.W.shape[0]
        assert self.banks % 2 == 1
        self.n_edge = (self.banks - 1) // 2
        self.open_cols = self.n_edge > 0 if open_cols is None else bool(open_cols)
        self.K, self.C, self.Lw = self.W.shape[-4], self.W.shape[-3], self.W.shape[-2]
        hshape = (self.K,) if self.W.ndim == 4 else (self.banks, self.K)
        self.hbias = np.ascontiguousarray(hbias, dtype=np.float32).reshape(hshape)
        self.vbias = np.ascontiguousarray(vbias, dtype=np.float32).reshape(self.C)
        self._p = _Params(self.K, self.C, self.Lw, self.W.ctypes.data, self.hbias.ctypes.data,
                          self.vbias.ctypes.data, int(self.open_cols), self.n_edge, 0)
        self.dense = False

    @property
    def p(self):
        return ct.byref(self._p)

    def n_hidden(self, L: int) -> int:
        return self.K * L * L


class FRBM:
    """Fully connected RBM of Sec. IV's comparison on an L x L lattice of C
    channels: W[K][C][L][L] (hidden unit k to every visible unit), hbias[K],
    vbias[C][L][L].  Drop-in for CRBM in the functions of this module."""

    def __init__(self, W, hbias, vbias):
        self.W = np.ascontiguousarray(W, dtype=np.float32)
        assert self.W.ndim == 4 and self.W.shape[2] == self.W.shape[3]
        self.K, self.C, self.Lw = self.W.shape[0], self.W.shape[1], self.W.shape[2]
        self.hbias = np.ascontiguousarray(hbias, dtype=np.float32).reshape(self.K)
        self.vbias = np.ascontiguousarray(vbias, dtype=np.float32).reshape(self.C, self.Lw, self.Lw)
        self.banks, self.n_edge, self.open_cols, self.dense = 1, 0, False, True
        self._p = _Params(self.K, self.C, self.Lw, self.W.ctypes.data, self.hbias.ctypes.data,
                          self.vbias.ctypes.data, 0, 0, 1)

    @property
    def p(self):
        return ct.byref(self._p)

    def n_hidden(self, L: int) -> int:
        assert L == self.Lw
        return self.K


# ---------------------------------------------------------------- RNG
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def mh_uniform(seed: int, t: int, g: int) -> float:
    return lib().orc_mh_uniform(seed, t, g)


def unit_uniform(seed: int, q: int, t: int, g: int, tag: int) -> float:
    return lib().orc_unit_uniform(seed, q, t, g, tag)


# ---------------------------------------------------------------- CRBM pieces
def hidden_preact(m: CRBM, v: np.ndarray, L: int) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.uint8).reshape(m.C, L, L)
    a = np.zeros((m.K,) if m.dense else (m.K, L, L), np.float64)
    lib().orc_hidden_preact(m.p, _ptr(v), L, _ptr(a))
    return a


def visible_preact(m: CRBM, h: np.ndarray, L: int) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=np.uint8).reshape((m.K,) if m.dense else (m.K, L, L))
    b = np.zeros((m.C, L, L), np.float64)
    lib().orc_visible_preact(m.p, _ptr(h), L, _ptr(b))
    return b


def free_energy(m: CRBM, x: np.ndarray) -> np.ndarray:
    """F of Eq. (free-energy_CRBM) for +-1 states x[B][C][L][L]."""
    x = np.ascontiguousarray(x, dtype=np.int8)
    B, L = x.shape[0], x.shape[-1]
    assert x.shape == (B, m.C, L, L)
    F = np.zeros(B, np.float64)
    lib().orc_free_energy(m.p, _ptr(x), B, L, _ptr(F))
    return F


def gibbs_step(m: CRBM, v: np.ndarray, L: int, seed: int, t: int, g: int, substep: int = 0):
    v = np.ascontiguousarray(v, dtype=np.uint8).reshape(m.C, L, L)
    h = np.zeros((m.K,) if m.dense else (m.K, L, L), np.uint8)
    vo = np.zeros((m.C, L, L), np.uint8)
    scratch = np.zeros(max(m.K, m.C) * L * L, np.float64)
    ties = lib().orc_gibbs_step(m.p, L, _ptr(v), _ptr(h), _ptr(vo), seed, t, g, substep, _ptr(scratch))
    return h, vo, ties


def grad(m: CRBM, x: np.ndarray, gF: np.ndarray):
    """sum_n gF[n] dF(x_n)/d(W, hbias, vbias), FP64."""
    x = np.ascontiguousarray(x, dtype=np.int8)
    B, L = x.shape[0], x.shape[-1]
    g = np.ascontiguousarray(gF, dtype=np.float64).reshape(B)
    dW = np.zeros(m.W.shape, np.float64)
    dhb = np.zeros(m.hbias.shape, np.float64)
    dvb = np.zeros(m.vbias.shape, np.float64)
    lib().orc_grad(m.p, _ptr(x), B, L, _ptr(g), _ptr(dW), _ptr(dhb), _ptr(dvb))
    return dW, dhb, dvb


# ---------------------------------------------------------------- targets
def ising_energy(s: np.ndarray, open_cols: bool = False) -> int:
    s = np.ascontiguousarray(s, dtype=np.int8)
    L = s.shape[-1]
    return int(lib().orc_ising_energy(_ptr(s), L, int(open_cols)))


def magnetization(s: np.ndarray) -> int:
    s = np.ascontiguousarray(s, dtype=np.int8)
    return int(lib().orc_magnetization(_ptr(s), s.shape[-1]))


def kitaev_matrix(u: np.ndarray, J=(1.0, 1.0, 1.0), open_cols: bool = False) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.int8)
    C, L = u.shape[0], u.shape[-1]
    Jv = np.ascontiguousarray(J, dtype=np.float64)
    M = np.zeros((L * L, L * L), np.float64)
    lib().orc_kitaev_matrix(_ptr(u), C, L, _ptr(Jv), int(open_cols), _ptr(M))
    return M


def singular_values(A: np.ndarray):
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    N = A.shape[0]
    sv = np.zeros(N, np.float64)
    sweeps = lib().orc_singular_values(_ptr(A), N, _ptr(sv))
    return sv, sweeps


def kitaev_S(u: np.ndarray, T: float, J=(1.0, 1.0, 1.0), open_cols: bool = False):
    """(S = -beta F, eps, E_f, C_f) of one gauge configuration u[C][L][L]."""
    u = np.ascontiguousarray(u, dtype=np.int8)
    C, L = u.shape[0], u.shape[-1]
    Jv = np.ascontiguousarray(J, dtype=np.float64)
    eps = np.zeros(L * L, np.float64)
    Ef = ct.c_double()
    Cf = ct.c_double()
    S = lib().orc_kitaev_S(_ptr(u), C, L, _ptr(Jv), int(open_cols), 1.0 / T, _ptr(eps), ct.byref(Ef),
                           ct.byref(Cf))
    return S, eps, Ef.value, Cf.value


def target(kind: int, x: np.ndarray, T=None, J=(1.0, 1.0, 1.0), boundary: int = 0):
    x = np.ascontiguousarray(x, dtype=np.int8)
    B, C, L = x.shape[0], x.shape[1], x.shape[-1]
    Jv = np.ascontiguousarray(J, dtype=np.float64)
    if kind == ISING:
        E = np.zeros(B, np.int64)
        lib().orc_target(0, _ptr(x), C, B, L, int(boundary), _ptr(Jv), None, _ptr(E), None)
        return E
    Tv = np.ascontiguousarray(T, dtype=np.float64).reshape(B)
    S = np.zeros(B, np.float64)
    lib().orc_target(1, _ptr(x), C, B, L, int(boundary), _ptr(Jv), _ptr(Tv), None, _ptr(S))
    return S


# ---------------------------------------------------------------- chains
def init_state(seed: int, n: int, C: int, L: int, g0: int = 0) -> np.ndarray:
    s = np.zeros((n, C, L, L), np.int8)
    lib().orc_init_state(seed, g0, n, C, L, _ptr(s))
    return s


def pt_uniform(seed: int, r: int, g: int) -> float:
    return float(lib().orc_pt_uniform(seed, r, g))


class Chains:
    """n independent chains of the CRBM-proposal + MH sampler (FP64).

    replica=True gives every chain a persistent CRBM replica (exchange
    correction); its initial state is a copy of the chain's (or `rbm_state`).
    tempering_swap() does one round of temperature swaps on the ladder grid
    chain = rung * n_ladders + ladder.  ties[0]: Gibbs near-ties, ties[1]: MH
    near-ties, ties[2]: swap near-ties."""

    def __init__(self, m: CRBM, target_kind: int, L: int, T, seed: int = 0, gibbs_k: int = 1,
                 burnin: int = 0, J=(1.0, 1.0, 1.0), state=None, g0: int = 0, replica: bool = False,
                 rbm_state=None, boundary: int = 0):
        self.m = m
        self.L = L
        self.T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
        n = self.T.shape[0]
        self.state = (init_state(seed, n, m.C, L, g0) if state is None
                      else np.array(state, dtype=np.int8, order="C", copy=True))
        assert self.state.shape == (n, m.C, L, L)
        self.rbm = None
        if replica or rbm_state is not None:
            self.rbm = (self.state.copy() if rbm_state is None
                        else np.array(rbm_state, dtype=np.int8, order="C", copy=True))
            assert self.rbm.shape == self.state.shape
        self.desc = _RunDesc(target_kind, L, n, gibbs_k, burnin, g0, seed, (ct.c_double * 3)(*J), int(boundary))
        self.rec = np.zeros(n, CHAIN_DTYPE)
        self.eps = np.zeros((n, L * L), np.float64) if target_kind == 1 else None
        self.t = 0
        self.ties = np.zeros(3, np.int64)
        lib().orc_chain_init(m.p, ct.byref(self.desc), _ptr(self.T), _ptr(self.state), _ptr(self.rec),
                             _ptr(self.eps) if self.eps is not None else None)

    def run(self, n_sweeps: int, log_accepts: bool = False, log_energy: bool = False):
        """Advance every chain n_sweeps.  Returns the accept log [n, n_sweeps]
        (or None); with log_energy the energy after each sweep (Ising E/J,
        Kitaev E_f) is left in self.energy_log [n, n_sweeps]."""
        n = self.T.shape[0]
        acc = np.zeros((n, n_sweeps), np.uint8) if log_accepts else None
        elog = np.zeros((n, n_sweeps), np.float64) if log_energy else None
        lib().orc_run(self.m.p, ct.byref(self.desc), _ptr(self.T), _ptr(self.state),
                      _ptr(self.rbm) if self.rbm is not None else None,
                      _ptr(self.eps) if self.eps is not None else None, self.t, n_sweeps,
                      _ptr(self.rec), _ptr(self.ties), _ptr(acc) if acc is not None else None,
                      _ptr(elog) if elog is not None else None)
        self.t += n_sweeps
        self.energy_log = elog
        return acc

    def tempering_swap(self, n_ladders: int, round_: int):
        n = self.T.shape[0]
        assert n % n_ladders == 0
        tie = np.zeros(1, np.int64)
        lib().orc_tempering_swap(ct.byref(self.desc), self.m.C, _ptr(self.T), _ptr(self.state), _ptr(self.rec),
                                 _ptr(self.eps) if self.eps is not None else None, n_ladders, round_, _ptr(tie))
        self.ties[2] += tie[0]


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops over chains (timing of the CPU baseline)."""
    lib().orc_set_threads(int(n))
