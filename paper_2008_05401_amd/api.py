"""Python interface of the CRBM sampler on MI355X.

torch provides device memory and the stream; every step of the sampler runs in
the HIP kernels of libcrbm.so (see include/crbm.h for the operations and
their paper references).
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as C
from . import autotune as _autotune

ISING, KITAEV, GIBBS = C.CRBM_ISING, C.CRBM_KITAEV, C.CRBM_GIBBS

# tile choices measured by the autotuner for this device (speed only)
_autotune.apply()


def set_tuning(L: int, K: int, Lw: int, rows: int, threads: int):
    C.crbm_set_tuning(L, K, Lw, rows, threads)


def clear_tuning():
    C.crbm_clear_tuning()


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev(device=None):
    return torch.device(device if device is not None else "cuda")


class CRBMParams:
    """Filters W[K][C][Lw][Lw], hbias[K], vbias[C] as float32 device tensors.

    The locally connected CRBM of Sec. IV.B passes W[1+2n][K][C][Lw][Lw] and
    hbias[1+2n][K] (bank 0 for the bulk hidden columns, banks 1..n for the
    left columns 0..n-1, banks n+1..2n for the right columns L-n..L-1);
    open_cols (default: on when there are edge banks) stops the filter windows
    at the column edge.

    dense=True makes it the fully connected RBM of the Sec. IV comparison:
    W[K][C][L][L] connects hidden unit k to every visible unit of an L x L
    lattice, hbias[K], vbias[C][L][L]."""

    def __init__(self, W, hbias, vbias, device=None, open_cols=None, dense: bool = False):
        dev = _dev(device)
        self.W = torch.as_tensor(np.asarray(W, np.float32) if not torch.is_tensor(W) else W,
                                 dtype=torch.float32, device=dev).contiguous()
        assert self.W.dim() in (4, 5) and self.W.shape[-1] == self.W.shape[-2]
        self.dense = bool(dense)
        assert not (self.dense and self.W.dim() != 4)
        self.banks = 1 if self.W.dim() == 4 else int(self.W.shape[0])
        assert self.banks % 2 == 1
        self.n_edge = (self.banks - 1) // 2
        self.open_cols = self.n_edge > 0 if open_cols is None else bool(open_cols)
        self.K, self.C, self.Lw = int(self.W.shape[-4]), int(self.W.shape[-3]), int(self.W.shape[-1])
        hshape = (self.K,) if self.W.dim() == 4 else (self.banks, self.K)
        self.hbias = torch.as_tensor(np.asarray(hbias, np.float32) if not torch.is_tensor(hbias) else hbias,
                                     dtype=torch.float32, device=dev).contiguous().reshape(hshape)
        self.vbias = torch.as_tensor(np.asarray(vbias, np.float32) if not torch.is_tensor(vbias) else vbias,
                                     dtype=torch.float32, device=dev).contiguous()
        self.vbias = self.vbias.reshape((self.C, self.Lw, self.Lw) if self.dense else (-1,))
        assert self.vbias.numel() == (self.C * self.Lw * self.Lw if self.dense else self.C)

    @classmethod
    def from_filters(cls, f, device=None, open_cols=None, dense: bool = False):
        return cls(f.W, f.hbias, f.vbias, device, open_cols, dense)

    def struct(self) -> C.crbm_params:
        return C.crbm_params(self.K, self.C, self.Lw, self.W.data_ptr(), self.hbias.data_ptr(),
                             self.vbias.data_ptr(), int(self.open_cols), self.n_edge, int(self.dense))


class Job:
    """n independent chains of the CRBM-proposal + MH sampler, resident on the GPU.

    replica=True (or an explicit rbm_state) gives every chain a persistent CRBM
    replica exchanged with the physical state each sweep (App. B exchange
    correction); without it the replica is refreshed from the physical state.
    tempering_swap() performs one round of temperature swaps on the ladder grid
    chain = rung * n_ladders + ladder.  mh_band_min widens the band of
    |log r - log u| inside which an MH decision is taken again on the exact
    route (a huge value sends every decision there)."""

    def __init__(self, params: CRBMParams, target: int, L: int, T, seed: int = 0, gibbs_k: int = 1,
                 burnin: int = 0, J=(1.0, 1.0, 1.0), state=None, chain_offset: int = 0, stream=None,
                 replica: bool = False, rbm_state=None, boundary: int = 0, mh_band_min: float = 0.0):
        dev = params.W.device
        self.params = params
        self.target = int(target)
        self.L = int(L)
        if torch.is_tensor(T) and T.device == dev:
            # a device tensor is used as it is (no host round trip)
            self.T = T.to(torch.float64).reshape(-1).contiguous()
        else:
            self.T = torch.as_tensor(np.asarray(T, np.float64).reshape(-1), device=dev).contiguous()
        n = int(self.T.numel())
        self.n_chains = n
        shape = (n, params.C, self.L, self.L)
        if state is None:
            self.state = torch.empty(shape, dtype=torch.int8, device=dev)
            init = 1
        else:
            st = state if torch.is_tensor(state) else torch.from_numpy(np.ascontiguousarray(state, np.int8))
            self.state = st.to(device=dev, dtype=torch.int8).contiguous().clone()
            assert tuple(self.state.shape) == shape
            init = 0
        self.rbm_state = None
        if replica or rbm_state is not None:
            if rbm_state is None:
                # filled by crbm_init (copy of the initial state) or copied from `state`
                self.rbm_state = (torch.empty(shape, dtype=torch.int8, device=dev) if init
                                  else self.state.clone())
            else:
                rs = rbm_state if torch.is_tensor(rbm_state) else torch.from_numpy(
                    np.ascontiguousarray(rbm_state, np.int8))
                self.rbm_state = rs.to(device=dev, dtype=torch.int8).contiguous().clone()
                assert tuple(self.rbm_state.shape) == shape
        self._p = params.struct()
        self._stream = stream
        self._desc = C.crbm_batch_desc(self.target, self.L, n, int(gibbs_k), int(burnin), init,
                                       int(chain_offset), int(boundary), int(seed), (C.ct.c_double * 3)(*J),
                                       self.T.data_ptr(), self.state.data_ptr(),
                                       self.rbm_state.data_ptr() if self.rbm_state is not None else None, 0, 0,
                                       float(mh_band_min))
        ws = C.crbm_workspace_size(self._p, self._desc)
        if ws == 0:
            # let crbm_init produce the precise error message
            ws = 256
        self.workspace = torch.zeros(ws + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._desc.workspace = aligned
        self._desc.workspace_bytes = ws + 256 - (aligned - base)
        self.ctx = C.crbm_init(self._p, self._desc, _stream_ptr(stream))

    def run(self, n_sweeps: int):
        C.crbm_propose_accept(self.ctx, int(n_sweeps))
        return self

    def tempering_swap(self, n_ladders: int, round_: int):
        C.crbm_tempering_swap(self.ctx, int(n_ladders), int(round_))
        return self

    def record_trace(self, length: int):
        """Keep the energy after each sweep (Ising E/J, Kitaev E_f) of every chain
        in a device ring buffer of `length` sweeps; 0 switches recording off."""
        length = int(length)
        if length <= 0:
            C.crbm_set_trace(self.ctx, None, 0)
            self._trace = None
            return self
        self._trace = torch.zeros((self.n_chains, length), dtype=torch.float64, device=self.state.device)
        self._trace_from = self.sweeps
        C.crbm_set_trace(self.ctx, self._trace.data_ptr(), length)
        return self

    def trace_ring(self):
        """(ring buffer [n_chains, length], start, count): the recorded energies
        in time order are ring[:, (start + i) % length] for i < count."""
        length = int(self._trace.shape[1])
        done = self.sweeps
        count = min(done - self._trace_from, length)
        return self._trace, (done - count) % length, count

    def trace(self) -> torch.Tensor:
        """Recorded energies in time order, [n_chains, count]."""
        ring, start, count = self.trace_ring()
        idx = (torch.arange(count, device=ring.device) + start) % ring.shape[1]
        return ring[:, idx]

    @property
    def sweeps(self) -> int:
        return C.crbm_sweeps_done(self.ctx)

    def stats(self) -> np.ndarray:
        out = np.zeros(self.n_chains, C.STATS_DTYPE)
        C.crbm_read_stats(self.ctx, out.ctypes.data, False)
        return out

    def stats_device(self) -> torch.Tensor:
        out = torch.empty(self.n_chains * C.STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.state.device)
        C.crbm_read_stats(self.ctx, out.data_ptr(), True)
        return out

    def close(self):
        if getattr(self, "ctx", None):
            C.crbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_many(jobs, n_sweeps: int):
    """Advance several jobs (same stream) by n_sweeps in shared launches."""
    C.crbm_propose_accept_many([j.ctx for j in jobs], int(n_sweeps))


class SweepGraph:
    """n_blocks blocks of sweeps_per_block sweeps of one or several jobs (same
    stream), captured once as a HIP graph and replayed by launch(); each launch
    advances the jobs exactly as run_many(jobs, sweeps_per_block) called
    n_blocks times would.  Holds the jobs, which must stay open while it lives."""

    def __init__(self, jobs, n_blocks: int, sweeps_per_block: int):
        self.jobs = list(jobs)
        self.sweeps = int(n_blocks) * int(sweeps_per_block)
        self.graph = C.crbm_graph_create([j.ctx for j in self.jobs], int(n_blocks), int(sweeps_per_block))

    def launch(self):
        if not self.graph:
            raise RuntimeError("graph is closed")
        if any(j.ctx is None for j in self.jobs):
            raise RuntimeError("a job of this graph has been closed")
        C.crbm_graph_launch(self.graph)
        return self

    def close(self):
        if getattr(self, "graph", None):
            C.crbm_graph_destroy(self.graph)
            self.graph = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autocorrelation(series: torch.Tensor, max_lag: int, c_window: float = 6.0, start: int = 0, stream=None):
    """Autocovariance C(t), t = 0..max_lag, integrated autocorrelation time and
    its automatic window for every row of `series` ([n, len] FP64 on the GPU;
    row g read as series[g, (start + i) % len]).  Returns (C [n, max_lag+1],
    tau [n], window [n]; window -1 where no lag up to max_lag qualifies)."""
    s = series.to(dtype=torch.float64).contiguous()
    n, ln = int(s.shape[0]), int(s.shape[1])
    out = torch.empty((n, int(max_lag) + 1), dtype=torch.float64, device=s.device)
    tau = torch.empty(n, dtype=torch.float64, device=s.device)
    win = torch.empty(n, dtype=torch.int32, device=s.device)
    C.crbm_autocorr(s.data_ptr(), n, ln, int(start), int(max_lag), float(c_window), out.data_ptr(), tau.data_ptr(),
                    win.data_ptr(), _stream_ptr(stream))
    return out, tau, win


def free_energy(params: CRBMParams, x: torch.Tensor, stream=None) -> torch.Tensor:
    x = x.to(device=params.W.device, dtype=torch.int8).contiguous()
    B, L = int(x.shape[0]), int(x.shape[-1])
    F = torch.empty(B, dtype=torch.float64, device=x.device)
    C.crbm_free_energy(params.struct(), x.data_ptr(), B, L, F.data_ptr(), _stream_ptr(stream))
    return F


def ising_energy(x: torch.Tensor, stream=None, boundary: int = 0) -> torch.Tensor:
    x = x.to(dtype=torch.int8).contiguous()
    B, L = int(x.shape[0]), int(x.shape[-1])
    E = torch.empty(B, dtype=torch.int32, device=x.device)
    C.target_energy(ISING, x.data_ptr(), B, 1, L, boundary, (1.0, 1.0, 1.0), None, E.data_ptr(), None,
                    _stream_ptr(stream))
    return E


def kitaev_weight(u: torch.Tensor, T, J=(1.0, 1.0, 1.0), stream=None, boundary: int = 0) -> torch.Tensor:
    u = u.to(dtype=torch.int8).contiguous()
    B, Cc, L = int(u.shape[0]), int(u.shape[1]), int(u.shape[-1])
    Tt = torch.as_tensor(np.asarray(T, np.float64).reshape(-1), device=u.device).contiguous()
    assert Tt.numel() == B
    S = torch.empty(B, dtype=torch.float64, device=u.device)
    C.target_energy(KITAEV, u.data_ptr(), B, Cc, L, boundary, J, Tt.data_ptr(), None, S.data_ptr(),
                    _stream_ptr(stream))
    return S


def grad(params: CRBMParams, x: torch.Tensor, gF: torch.Tensor, stream=None):
    """sum_b gF[b] dF(x_b)/d(W, hbias, vbias) as float32 device tensors."""
    x = x.to(device=params.W.device, dtype=torch.int8).contiguous()
    B, L = int(x.shape[0]), int(x.shape[-1])
    g = gF.to(device=x.device, dtype=torch.float32).contiguous().reshape(B)
    p = params.struct()
    ws_bytes = C.crbm_grad_workspace_size(p, B)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=x.device)
    dW = torch.empty_like(params.W)
    dhb = torch.empty_like(params.hbias)
    dvb = torch.empty_like(params.vbias)
    C.crbm_grad(p, x.data_ptr(), B, L, g.data_ptr(), dW.data_ptr(), dhb.data_ptr(), dvb.data_ptr(),
                ws.data_ptr(), ws_bytes, _stream_ptr(stream))
    return dW, dhb, dvb


def grad_static(params: CRBMParams, x: torch.Tensor, gF: torch.Tensor, stream=None):
    """As grad(), through crbm_grad_static: no workspace, the library's static
    scratch (at most 8 MiB of partial gradients; calls on one GPU must not
    overlap).  The outputs are the caller's tensors, allocated here."""
    x = x.to(device=params.W.device, dtype=torch.int8).contiguous()
    B, L = int(x.shape[0]), int(x.shape[-1])
    g = gF.to(device=x.device, dtype=torch.float32).contiguous().reshape(B)
    dW = torch.empty_like(params.W)
    dhb = torch.empty_like(params.hbias)
    dvb = torch.empty_like(params.vbias)
    C.crbm_grad_static(params.struct(), x.data_ptr(), B, L, g.data_ptr(), dW.data_ptr(), dhb.data_ptr(),
                       dvb.data_ptr(), _stream_ptr(stream))
    return dW, dhb, dvb


class CRBMFreeEnergy(torch.autograd.Function):
    """F(x; W, hbias, vbias) with the hand-written backward kernel.

    forward(x, W, hbias, vbias) -> F[B] (float64); backward returns
    (None, dW, dhbias, dvbias) with d = sum_b grad_out[b] dF_b/dtheta."""

    @staticmethod
    def forward(ctx, x, W, hbias, vbias, open_cols=None, dense=False):
        p = CRBMParams(W.detach(), hbias.detach(), vbias.detach(), device=W.device, open_cols=open_cols, dense=dense)
        ctx.save_for_backward(x, W, hbias, vbias)
        ctx.open_cols, ctx.dense = open_cols, dense
        return free_energy(p, x)

    @staticmethod
    def backward(ctx, gout):
        x, W, hbias, vbias = ctx.saved_tensors
        p = CRBMParams(W.detach(), hbias.detach(), vbias.detach(), device=W.device, open_cols=ctx.open_cols,
                       dense=ctx.dense)
        dW, dhb, dvb = grad(p, x, gout.to(torch.float32))
        return None, dW, dhb.reshape(hbias.shape), dvb.reshape(vbias.shape), None, None


def crbm_free_energy_fn(x, W, hbias, vbias, open_cols=None, dense=False):
    return CRBMFreeEnergy.apply(x, W, hbias, vbias, open_cols, dense)
