"""Training of a CRBM (Alg. 1 "Train the RBM") and transfer to a larger
lattice, on the GPU, for the Ising and the Kitaev targets.

* Loss of Eq. (loss) with the optimal constant C(W): for a minibatch,
  diff_i = nlp(x_i) - F(x_i) with nlp = -log P_phys up to a constant
  (beta E for Ising, -S for Kitaev), C = mean(diff), loss = mean((diff - C)^2),
  minimised with ADAM; F and its gradient run in the HIP kernels through
  `api.CRBMFreeEnergy` (forward `crbm_free_energy`, backward `crbm_grad`).
* Parameters initialised as in Alg. 1: W ~ N(0, 2/(K Lw^2)), biases 0.
* Replay buffer of RBM samples (Alg. 1): `ub` persistent block-Gibbs chains
  of the current CRBM (target CRBM_GIBBS) started from Binomial(p = 0.5)
  states; each buffer update advances them by k Gibbs steps and puts them in
  front of x_RBM, the oldest states dropped beyond the train size N; the
  buffer is filled to N before training; the nlp of new states is evaluated on
  the GPU.
* Physical training states:
  - Ising: independent chains of the exact sampler (the App. C kernel of the
    target temperature plus the MH correction), so no local Metropolis run is
    needed (Sec. III notes the same for the Ising case);
  - Kitaev (Sec. IV, pre-training): the CRBM is first trained on uniformly
    random gauge configurations with their exact weights, then samples of the
    physical distribution are drawn with the pre-trained CRBM through the
    exchange-corrected sampler and the training is finished on them.
* Open boundaries (Sec. IV.B): the locally connected CRBM starts from the
  filters of a periodic CRBM (every bank a copy) and is retrained on samples
  of the open-boundary target drawn with itself.
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


def ising_nlp(T: float):
    """-log P of the Ising model at T up to a constant: beta E (J = 1)."""
    return lambda x: api.ising_energy(x).to(torch.float64) / T


def kitaev_nlp(T: float, J=(1.0, 1.0, 1.0), boundary: int = 0):
    """-log P of the Kitaev gauge field at T up to a constant: -S."""
    return lambda x: -api.kitaev_weight(x, np.full(int(x.shape[0]), T), J, boundary=boundary)


@dataclass
class TrainResult:
    W: torch.Tensor
    hbias: torch.Tensor
    vbias: torch.Tensor
    losses: list
    steps: int
    # the replay buffer x_RBM at the end and its -log P_phys (None without replay)
    x_rbm: torch.Tensor = None
    nlp_rbm: torch.Tensor = None
    # per epoch (with track=True): the loss of Eq. (loss) with its optimal C over
    # the epoch's training set x_tot = x_phys U x_RBM before and after the epoch's
    # steps, and after them over x_phys and over x_RBM alone; "offset" is the mean
    # of E beta - F over x_RBM minus that over x_phys (after the steps)
    history: list = None
    # with keep_best: the epoch whose parameters are returned
    best_epoch: int = None


def _params_of(f, dev):
    return (torch.tensor(f.W, device=dev, requires_grad=True), torch.tensor(f.hbias, device=dev, requires_grad=True),
            torch.tensor(f.vbias, device=dev, requires_grad=True))


def _loss_over(x, nlp, W, hb, vb, open_cols):
    with torch.no_grad():
        F = api.crbm_free_energy_fn(x, W, hb, vb, open_cols)
        d = nlp - F
        return float(((d - d.mean()) ** 2).mean()), float(d.mean())


def train_crbm(x_phys: torch.Tensor, nlp_phys: torch.Tensor, nlp_fn, T: float, K: int = 8, Lw: int = 5,
               epochs: int = 30, batch: int = 20, lr: float = 1e-3, ub: int = 200, gibbs_k: int = 1, seed: int = 0,
               train_size: int = None, log_every: int = 0, init=None, replay: bool = True,
               open_cols=None, track: bool = False, keep_best: bool = False) -> TrainResult:
    """Alg. 1 on physical states x_phys [n][C][L][L] with nlp_phys = -log P(x_phys) + const.
    `nlp_fn(x)` evaluates the same for replay-buffer states; `init` optionally
    continues from filters (W, hbias, vbias) instead of the Alg. 1 initialisation
    (filter banks of a locally connected CRBM included; open_cols as in
    api.CRBMParams).  The buffer x_RBM is filled to the train size N before the
    first epoch (Alg. 1 iterates UPDATE BUFFER until its size is N); every epoch
    then runs UPDATE BUFFER once and one pass of minibatches over x_phys U x_RBM.
    Training stops when the loss no longer decreases (App. D); with keep_best the
    parameters returned are those of the epoch whose loss over its x_tot, after
    its steps, was lowest (ADAM at batch 20 leaves the loss fluctuating around
    its floor from epoch to epoch)."""
    dev = x_phys.device
    C = int(x_phys.shape[1])
    L = int(x_phys.shape[-1])
    if init is None:
        f0 = workloads.alg1_init_filters(K, Lw, seed=seed, C=C)
        W, hb, vb = _params_of(f0, dev)
    else:
        W, hb, vb = (t.detach().clone().to(dev).requires_grad_(True) for t in init)
    opt = torch.optim.Adam([W, hb, vb], lr=lr)
    N = train_size or int(x_phys.shape[0])
    gen = torch.Generator(device="cpu").manual_seed(seed)
    nlp_phys = nlp_phys.to(device=dev, dtype=torch.float64)
    xb = nb = None
    if replay and ub < 1:
        raise ValueError(f"the buffer update size ub must be >= 1 (got {ub})")
    if replay:
        # x-bar_RBM starts from Binomial(p = 0.5) states (Alg. 1)
        chains = torch.from_numpy(workloads.random_states(ub, C, L, seed=seed + 1)).to(dev)
        xb = chains[:0]
        nb = torch.zeros(0, dtype=torch.float64, device=dev)
        n_upd = 0

        def update_buffer():
            # UPDATE BUFFER: k Gibbs steps of the current CRBM on x-bar_RBM, which joins
            # x_RBM in front; the oldest states beyond N are removed
            nonlocal chains, xb, nb, n_upd
            p = api.CRBMParams(W.detach(), hb.detach(), vb.detach(), device=dev, open_cols=open_cols)
            job = api.Job(p, api.GIBBS, L, np.full(ub, T), seed=seed + 1000 + n_upd, gibbs_k=gibbs_k, state=chains)
            job.run(1)
            chains = job.state.clone()
            job.close()
            n_upd += 1
            xb = torch.cat([chains, xb])[:N]
            nb = torch.cat([nlp_fn(chains).to(torch.float64), nb])[:N]

        while xb.shape[0] < N:
            update_buffer()
    losses = []
    history = [] if track else None
    best = None
    steps = 0
    for ep in range(epochs):
        if replay:
            update_buffer()
            x_tot = torch.cat([x_phys, xb])
            n_tot = torch.cat([nlp_phys, nb])
        else:
            x_tot, n_tot = x_phys, nlp_phys
        if track:
            before, _ = _loss_over(x_tot, n_tot, W, hb, vb, open_cols)
        perm = torch.randperm(x_tot.shape[0], generator=gen).to(dev)
        for s0 in range(0, x_tot.shape[0] - batch + 1, batch):
            idx = perm[s0:s0 + batch]
            F = api.crbm_free_energy_fn(x_tot[idx], W, hb, vb, open_cols)
            diff = n_tot[idx] - F
            Cc = diff.mean()
            loss = ((diff - Cc) ** 2).mean()
            opt.zero_grad(set_to_none=True)
            loss.backward()
            opt.step()
            steps += 1
            losses.append(float(loss.detach()) if (log_every and steps % log_every == 0) else math.nan)
        if track or keep_best:
            after, _ = _loss_over(x_tot, n_tot, W, hb, vb, open_cols)
            if keep_best and (best is None or after < best[0]):
                best = (after, ep, W.detach().clone(), hb.detach().clone(), vb.detach().clone())
        if track:
            lp, cp = _loss_over(x_phys, nlp_phys, W, hb, vb, open_cols)
            h = {"epoch": ep, "steps": steps, "loss_tot_before": before, "loss_tot_after": after, "loss_phys": lp}
            if replay:
                lr_, cr = _loss_over(xb, nb, W, hb, vb, open_cols)
                h.update(loss_rbm=lr_, offset=cr - cp)
            history.append(h)
    if best is not None:
        return TrainResult(best[2], best[3], best[4], losses, steps, xb, nb, history, best_epoch=best[1])
    return TrainResult(W.detach().clone(), hb.detach().clone(), vb.detach().clone(), losses, steps, xb, nb, history)


def train(x_phys: torch.Tensor, E_phys: torch.Tensor, T: float, **kw) -> TrainResult:
    """Alg. 1 for the Ising model: physical states with their energies E (J = 1)."""
    return train_crbm(x_phys, E_phys.to(torch.float64) / T, ising_nlp(T), T, **kw)


def full_loss(x: torch.Tensor, E: torch.Tensor, T: float, W, hb, vb) -> float:
    """The Ising loss of Eq. (loss) with its optimal constant over the whole set."""
    return full_loss_nlp(x, E.to(torch.float64) / T, W, hb, vb)


def full_loss_nlp(x: torch.Tensor, nlp: torch.Tensor, W, hb, vb, open_cols=None) -> float:
    """The loss of Eq. (loss) with its optimal constant over the whole set."""
    p = api.CRBMParams(W, hb, vb, device=W.device, open_cols=open_cols)
    F = api.free_energy(p, x)
    diff = nlp.to(torch.float64) - F
    return float(((diff - diff.mean()) ** 2).mean())


def union_loss(res: TrainResult, x_phys: torch.Tensor, nlp_phys: torch.Tensor, W, hb, vb, open_cols=None) -> float:
    """The quantity Alg. 1 minimises: the loss of Eq. (loss), optimal C, over
    x_phys U x_RBM with the replay buffer x_RBM that `res` ended with, for the
    parameters (W, hb, vb)."""
    x = torch.cat([x_phys, res.x_rbm])
    nlp = torch.cat([nlp_phys.to(torch.float64), res.nlp_rbm.to(torch.float64)])
    return full_loss_nlp(x, nlp, W, hb, vb, open_cols)


def kitaev_pretrain_and_train(L: int, T: float, K: int = 8, Lw: int = 3, n_random: int = 4096, n_phys: int = 512,
                              pre_epochs: int = 10, epochs: int = 10, sweeps: int = 200, lr: float = 1e-3,
                              seed: int = 0, J=(1.0, 1.0, 1.0)):
    """Sec. IV pre-training of a Kitaev CRBM (C = 3 bond channels): Alg. 1's loss
    on uniformly random gauge configurations, then physical samples drawn with
    the pre-trained CRBM (persistent replicas, exchange-corrected) and Alg. 1
    with the replay buffer on them.  Returns (pretrained, trained, physical
    samples, their exchange acceptance, the random pre-training states)."""
    dev = torch.device("cuda")
    nlp = kitaev_nlp(T, J)
    xr = torch.from_numpy(workloads.random_states(n_random, 3, L, seed=seed + 7)).to(dev)
    pre = train_crbm(xr, nlp(xr), nlp, T, K=K, Lw=Lw, epochs=pre_epochs, batch=64, lr=lr, seed=seed, replay=False)
    p = api.CRBMParams(pre.W, pre.hbias, pre.vbias, device=dev)
    job = api.Job(p, api.KITAEV, L, np.full(n_phys, T), seed=seed + 11, J=J, replica=True)
    done = 0
    while done < sweeps:
        b = min(50, sweeps - done)
        job.run(b)
        done += b
    x = job.state.clone()
    st = job.stats()
    acc = float(st["n_acc"].sum() / max(1, st["sweeps"].sum()))
    job.close()
    fin = train_crbm(x, nlp(x), nlp, T, K=K, Lw=Lw, epochs=epochs, batch=20, lr=lr, ub=128, seed=seed + 1,
                     init=(pre.W, pre.hbias, pre.vbias), track=True, keep_best=True)
    return pre, fin, x, acc, xr


def sample_states(params, target: int, L: int, T: float, n: int, sweeps: int, seed: int, J=(1.0, 1.0, 1.0),
                  boundary: int = 0):
    """n states of the physical target drawn by the exchange-corrected sampler
    (persistent CRBM replicas) after `sweeps` sweeps; returns (states,
    exchange acceptance)."""
    job = api.Job(params, target, L, np.full(n, T), seed=seed, J=J, replica=True, boundary=boundary)
    done = 0
    while done < sweeps:
        b = min(50, sweeps - done)
        job.run(b)
        done += b
    x = job.state.clone()
    st = job.stats()
    acc = float(st["n_acc"].sum() / max(1, st["sweeps"].sum()))
    job.close()
    return x, acc


def kitaev_open_transfer(periodic: TrainResult, L: int, T: float, n_edge: int = 3, n_phys: int = 256,
                         sweeps: int = 40, epochs: int = 6, lr: float = 1e-3, seed: int = 0, J=(1.0, 1.0, 1.0)):
    """Sec. IV.B: a locally connected CRBM for the open-boundary Kitaev target.
    Every filter bank starts as a copy of the periodic CRBM; samples of the
    open-boundary target at size L are drawn with it (exchange-corrected) and
    Alg. 1 retrains all banks on them.  Returns (initial LCRBM, retrained
    LCRBM, samples)."""
    dev = periodic.W.device
    nb = 1 + 2 * n_edge
    W0 = periodic.W.detach().unsqueeze(0).repeat(nb, 1, 1, 1, 1).contiguous()
    hb0 = periodic.hbias.detach().reshape(1, -1).repeat(nb, 1).contiguous()
    vb0 = periodic.vbias.detach().clone()
    init = TrainResult(W0, hb0, vb0, [], 0)
    p = api.CRBMParams(W0, hb0, vb0, device=dev)
    x, _ = sample_states(p, api.KITAEV, L, T, n_phys, sweeps, seed + 21, J=J, boundary=1)
    nlp = kitaev_nlp(T, J, boundary=1)
    fin = train_crbm(x, nlp(x), nlp, T, K=int(W0.shape[1]), Lw=int(W0.shape[-1]), epochs=epochs, batch=20, lr=lr,
                     ub=128, seed=seed + 3, init=(W0, hb0, vb0), track=True, keep_best=True)
    return init, fin, x
