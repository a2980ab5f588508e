"""Training of a CRBM on Ising samples (Alg. 1 "Train the RBM") and transfer to
a larger lattice, on the GPU.

* Physical training states: independent chains of the exact sampler (the
  App. C kernel of the target temperature plus the MH correction), so no
  local Metropolis run is needed (Sec. III notes the same for the Ising case).
* Parameters initialised as in Alg. 1: W ~ N(0, 2/(K Lw^2)), biases 0.
* Replay buffer of RBM samples (Alg. 1): `ub` new states per epoch from plain
  block-Gibbs chains of the current CRBM (target CRBM_GIBBS), the oldest
  states dropped beyond the train size.
* Loss of Eq. (loss) with the optimal constant C(W): for a minibatch,
  diff_i = beta E(x_i) - F(x_i), C = mean(diff), loss = mean((diff - C)^2),
  minimised with ADAM; F and its gradient run in the HIP kernels through
  `api.CRBMFreeEnergy` (forward `crbm_free_energy`, backward `crbm_grad`).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import api, workloads


def exact_ising_samples(L: int, T: float, n: int, sweeps: int = 1000, seed: int = 0, K: int = 8, Lw: int = 5):
    """n independent Ising states at temperature T: the exact CRBM kernels of
    App. C (zero-padded to K x Lw x Lw) as proposal, corrected by MH."""
    f = workloads.analytic_ising_filters(T, K=K, Lw=Lw)
    job = api.Job(api.CRBMParams.from_filters(f), api.ISING, L, np.full(n, T), seed=seed)
    done = 0
    while done < sweeps:
        b = min(100, sweeps - done)
        job.run(b)
        done += b
    st = job.stats()
    x = job.state.clone()
    E = api.ising_energy(x)
    return x, E, float(st["n_acc"].sum() / max(1, st["sweeps"].sum()))


@dataclass
class TrainResult:
    W: torch.Tensor
    hbias: torch.Tensor
    vbias: torch.Tensor
    losses: list
    steps: int


def train(x_phys: torch.Tensor, E_phys: torch.Tensor, T: float, K: int = 8, Lw: int = 5, epochs: int = 30,
          batch: int = 20, lr: float = 1e-3, ub: int = 200, gibbs_k: int = 1, seed: int = 0,
          train_size: int = None, log_every: int = 0) -> TrainResult:
    dev = x_phys.device
    L = int(x_phys.shape[-1])
    beta = 1.0 / T
    f0 = workloads.alg1_init_filters(K, Lw, seed=seed)
    W = torch.tensor(f0.W, device=dev, requires_grad=True)
    hb = torch.tensor(f0.hbias, device=dev, requires_grad=True)
    vb = torch.tensor(f0.vbias, device=dev, requires_grad=True)
    opt = torch.optim.Adam([W, hb, vb], lr=lr)
    N = train_size or int(x_phys.shape[0])
    gen = torch.Generator(device="cpu").manual_seed(seed)
    # buffer starts from Binomial(p = 0.5) states (Alg. 1)
    buf = torch.from_numpy(workloads.random_states(ub, 1, L, seed=seed + 1)).to(dev)
    xb = buf.clone()
    Eb = api.ising_energy(xb)
    losses = []
    steps = 0
    t_sweep = 0
    for ep in range(epochs):
        # UPDATE BUFFER: k Gibbs steps of the current CRBM from the previous new states
        p = api.CRBMParams(W.detach(), hb.detach(), vb.detach(), device=dev)
        job = api.Job(p, api.GIBBS, L, np.full(ub, T), seed=seed + 1000 + ep, gibbs_k=gibbs_k, state=buf)
        job.run(1)
        buf = job.state.clone()
        t_sweep += 1
        xb = torch.cat([buf, xb])[:N]
        Eb = torch.cat([api.ising_energy(buf), Eb])[:N]
        x_tot = torch.cat([x_phys, xb])
        E_tot = torch.cat([E_phys, Eb]).to(torch.float64)
        perm = torch.randperm(x_tot.shape[0], generator=gen).to(dev)
        for s0 in range(0, x_tot.shape[0] - batch + 1, batch):
            idx = perm[s0:s0 + batch]
            F = api.crbm_free_energy_fn(x_tot[idx], W, hb, vb)
            diff = beta * E_tot[idx] - F
            C = diff.mean()
            loss = ((diff - C) ** 2).mean()
            opt.zero_grad(set_to_none=True)
            loss.backward()
            opt.step()
            steps += 1
            losses.append(float(loss.detach()) if (log_every and steps % log_every == 0) else math.nan)
    return TrainResult(W.detach().clone(), hb.detach().clone(), vb.detach().clone(), losses, steps)


def full_loss(x: torch.Tensor, E: torch.Tensor, T: float, W, hb, vb) -> float:
    """The loss of Eq. (loss) with its optimal constant over the whole set."""
    p = api.CRBMParams(W, hb, vb, device=W.device)
    F = api.free_energy(p, x)
    diff = E.to(torch.float64) / T - F
    return float(((diff - diff.mean()) ** 2).mean())
