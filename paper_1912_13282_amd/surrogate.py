"""Training and use of the learned 2D Laplacian surrogate.

Host orchestration only: every arithmetic step (stencils, plain weights,
features, forward, backward, Adam, projection) runs in the HIP library.

    sets  = training_node_sets(count, seed0)          # jittered unit-disk node sets
    data  = build_training_set(sets)                  # features / targets on the GPU
    state = TrainState.init(seed)                     # Xavier-uniform weights, Adam moments
    train(state, data, epochs, batch, lr)             # Adam, cosine learning-rate decay
    w, st = surrogate_laplacian(X, offsets, idx, state.params)

Training pairs: for each stencil, the scaled offsets (x_j - x_i)/s in stencil
order and the plain FP64 RBF-FD Laplacian weights scaled by s^2 (PHS r^3,
degree-2 monomials, n = 15, eq. rbf-system-aug).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _binding as B

N_STENCIL = 15
DEGREE = 2


def training_node_sets(count: int, seed0: int = 4_000_000, h: float | None = None):
    """Seeded jittered unit-disk node sets (the 2D disk generator, seeds seed0 + k)."""
    import nodesets as ns
    return [ns.disk(h or ns.DISK_H, seed0 + k) for k in range(count)]


@dataclass
class TrainingSet:
    feat: torch.Tensor    # [S, 30] float32
    target: torch.Tensor  # [S, 15] float32 (w_lap * s^2)


def build_training_set(node_sets, device=None) -> TrainingSet:
    """Stencils (exact kNN), plain FP64 Laplacian weights and the training pairs, all on the GPU."""
    dev = torch.device(device or "cuda")
    feats, tgts = [], []
    for nd in node_sets:
        X = torch.from_numpy(np.ascontiguousarray(nd.X)).to(dev)
        N = X.shape[0]
        off = torch.arange(0, (N + 1) * N_STENCIL, N_STENCIL, dtype=torch.int64, device=dev)
        idx = B.select_stencils(X, off, N_STENCIL)
        w, st = B.compute_weights(X, off, idx, N_STENCIL, DEGREE, ("lap",), precision="f64")
        f, t, _ = B.surrogate_dataset(X, off, idx, w_lap=w[0])
        feats.append(f)
        tgts.append(t)
    return TrainingSet(torch.cat(feats), torch.cat(tgts))


@dataclass
class TrainState:
    params: torch.Tensor   # [MLP_NPARAM] float32 master weights
    m: torch.Tensor
    v: torch.Tensor
    packed: torch.Tensor   # bfloat16 operand copy of params
    step: int = 0

    @staticmethod
    def init(seed: int, device=None) -> "TrainState":
        import nodesets as ns
        dev = torch.device(device or "cuda")
        p = B.mlp_flatten({k: torch.from_numpy(v) for k, v in ns.surrogate_init(seed).items()}).to(dev)
        return TrainState.from_params(p)

    @staticmethod
    def from_params(p: torch.Tensor, step: int = 0) -> "TrainState":
        p = p.to(torch.float32).contiguous().clone()
        return TrainState(p, torch.zeros_like(p), torch.zeros_like(p), B.mlp_pack(p), step)

    def save(self, path: str):
        torch.save({"params": self.params.cpu(), "m": self.m.cpu(), "v": self.v.cpu(),
                    "step": torch.tensor(self.step)}, path)

    @staticmethod
    def load(path: str, device=None) -> "TrainState":
        dev = torch.device(device or "cuda")
        d = torch.load(path, map_location="cpu", weights_only=True)
        st = TrainState.from_params(d["params"].to(dev), int(d["step"]))
        st.m.copy_(d["m"].to(dev))
        st.v.copy_(d["v"].to(dev))
        return st


def cosine_lr(step: int, total: int, lr0: float, lr_min: float = 0.0) -> float:
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * min(step, total) / max(total, 1)))


def train(state: TrainState, data: TrainingSet, epochs: int, batch: int = 8192, lr: float = 1e-3,
          seed: int = 0, total_steps: int | None = None, log=None):
    """Adam on the mean-squared error, minibatches drawn by a seeded permutation per epoch."""
    S = data.feat.shape[0]
    dev = data.feat.device
    steps_per_epoch = S // batch
    total = total_steps or epochs * steps_per_epoch
    g = torch.Generator(device="cpu").manual_seed(seed)
    grads = torch.empty_like(state.params)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ws = torch.empty(B.mlp_grad_workspace(batch), dtype=torch.uint8, device=dev)
    history = []
    for ep in range(epochs):
        perm = torch.randperm(S, generator=g).to(dev)
        acc = torch.zeros((), dtype=torch.float64, device=dev)
        for k in range(steps_per_epoch):
            sel = perm[k * batch:(k + 1) * batch]
            B.mlp_grad(state.params, state.packed, data.feat, data.target, sel=sel, grads=grads, loss=loss,
                       workspace=ws)
            state.step += 1
            B.mlp_adam(state.params, grads, state.m, state.v, state.step, cosine_lr(state.step - 1, total, lr),
                       packed=state.packed)
            acc += loss[0]
        mean = float(acc) / max(steps_per_epoch, 1)
        history.append(mean)
        if log:
            log(f"epoch {ep}: loss {mean:.4e}")
    return history


def surrogate_laplacian(X, offsets, idx, params: torch.Tensor, n_max: int = N_STENCIL, tol: float = 1e-6,
                        corr_tol: float = 0.25):
    """Laplacian weights through the network + projection (plain solve where rejected;
    corr_tol = inf accepts every consistent projection, the ablation without the gate)."""
    B.surrogate_load(params)
    return B.surrogate_weights(X, offsets, idx, n_max, surrogate_tol=tol, surrogate_corr_tol=corr_tol)
