"""Training driver of the learned warm start (argument marshalling only: the
sketch, the network's forward and backward passes, the alignment loss and the
Adam step all run in the HIP library, see include/tucker_learn.h).

A training sample is one mode of one tensor: its sketch features (F, rho)
from ``learn_sketch`` and target factors A* (In x J, orthonormal columns,
float64 on the GPU), for example converged factors of a decomposition. One
Adam step uses one sample, cycling through them.
"""
from __future__ import annotations

import numpy as np

from . import (learn_adam, learn_align, learn_backward, learn_forward, learn_param_count, learn_sketch,
               learn_test_width)

N_IN, N_HID, N_OUT = 64, 128, 128
DEFAULT_SEED = 0x5EED


def init_params(seed: int = 0, device="cuda"):
    """He-scaled Gaussian weights, zero biases (float32 on the device). The
    second layer starts as a scaled identity plus noise, so that the network
    starts close to passing the rectified sketch features through."""
    import torch
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((N_IN, N_HID)) * np.sqrt(2.0 / N_IN)
    b1 = np.zeros(N_HID)
    W2 = np.eye(N_HID, N_OUT) + rng.standard_normal((N_HID, N_OUT)) * np.sqrt(0.1 / N_HID)
    b2 = np.zeros(N_OUT)
    theta = np.concatenate([W1.ravel(), b1, W2.ravel(), b2]).astype(np.float32)
    assert theta.size == learn_param_count()
    return torch.from_numpy(theta).to(device)


def make_sample(idx, vals, dims, mode: int, target, seed: int = DEFAULT_SEED):
    """(F, rho, A*, K) for one mode of one tensor (all on the GPU); K is the
    test width of the target's rank."""
    import torch
    F, rho = learn_sketch(idx, vals, dims, mode, seed)
    A = torch.as_tensor(target, dtype=torch.float64).to(vals.device).contiguous()
    return F, rho, A, learn_test_width(int(A.shape[1]))


def sample_loss(params, sample, shift=1e-6) -> float:
    F, rho, A, K = sample
    R, _ = learn_forward(F, rho, params, want_z1=False)
    return learn_align(R, K, A, shift, want_grad=False)[0]


def train(params, samples, steps: int = 300, lr: float = 3e-3, shift: float = 1e-6, log_every: int = 0, log=print):
    """Adam on the subspace-alignment loss, one sample per step. Updates
    `params` in place and returns the per-step losses."""
    import torch
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    losses = []
    for step in range(1, steps + 1):
        F, rho, A, K = samples[(step - 1) % len(samples)]
        R, Z1 = learn_forward(F, rho, params)
        loss, dR = learn_align(R, K, A, shift)
        g = learn_backward(F, rho, params, Z1, dR)
        learn_adam(params, g, m, v, step, lr=lr)
        losses.append(loss)
        if log_every and step % log_every == 0:
            k = min(len(samples), step)
            log(f"step {step}: mean loss over the last {k} samples {np.mean(losses[-k:]):.4f}")
    return losses
