"""Warm-start surrogate: a four-layer dilated 3x3 convolution network on a
k-coarsened grid that predicts a steady force-driven channel flow past
obstacles, trained on steady fields the lattice solver produces, and used to
initialise new solves (f = f_eq(rho, u) + f_ne with f_ne from the predicted
velocity gradient, Sec. IV eq. fne).

Orchestration only: every arithmetic step (convolutions and their gradients,
loss, Adam, features, targets, initial fields, lattice steps, residuals)
runs in librmrt.so kernels; torch provides device memory and the stream.

Network: channels 16 -> 32 -> 32 -> 32 -> 16 (inputs: solid fraction,
Poiseuille prior, Re; outputs: u/Ut - prior, v/Ut, (rho - 1) * 100; the rest
are zero padding), dilations 1, 2, 4, 8 (receptive field 31 coarse cells),
SiLU between layers, bf16 weights and activations, fp32 accumulation, master
weights and Adam state in fp32.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import rmrt as R

CHANS = (16, 32, 32, 32, 16)
DILS = (1, 2, 4, 8)
COARSEN = 4
RE_SCALE = 100.0
RHO_SCALE = 100.0


class Surrogate:
    """Parameters, Adam state and activation buffers for batches of B images of H x W."""

    def __init__(self, seed=0, B=16, H=64, W=128, device="cuda"):
        rng = np.random.default_rng(seed)
        self.dils = DILS
        self.B, self.H, self.W = B, H, W
        self.w32, self.wbf, self.b32, self.gw, self.gb = [], [], [], [], []
        self.mw, self.vw, self.mb, self.vb, self.wt = [], [], [], [], []
        for l in range(4):
            ci, co = CHANS[l], CHANS[l + 1]
            scale = math.sqrt(2.0 / (9 * ci)) * (0.1 if l == 3 else 1.0)
            w = torch.tensor(rng.standard_normal((co, 3, 3, ci)) * scale, dtype=torch.float32, device=device)
            self.w32.append(w)
            wb = torch.empty(w.shape, dtype=torch.bfloat16, device=device)
            R.nn_to_bf16(w, wb)
            self.wbf.append(wb)
            self.b32.append(torch.zeros(co, dtype=torch.float32, device=device))
            self.gw.append(torch.zeros_like(w))
            self.gb.append(torch.zeros(co, dtype=torch.float32, device=device))
            self.mw.append(torch.zeros_like(w))
            self.vw.append(torch.zeros_like(w))
            self.mb.append(torch.zeros(co, dtype=torch.float32, device=device))
            self.vb.append(torch.zeros(co, dtype=torch.float32, device=device))
            self.wt.append(torch.empty((ci, 3, 3, co), dtype=torch.bfloat16, device=device))
        self.t = 0
        self._alloc(B, H, W, device)

    def _alloc(self, B, H, W, device):
        self.B, self.H, self.W = B, H, W
        self.a = [torch.empty((B, H, W, c), dtype=torch.bfloat16, device=device) for c in CHANS[:4]]
        self.y = [torch.empty((B, H, W, c), dtype=torch.float32, device=device) for c in CHANS[1:]]
        self.g = [torch.empty((B, H, W, c), dtype=torch.bfloat16, device=device) for c in CHANS[1:]]
        need = max(R.nn_wgrad_scratch_floats(B, H, W, CHANS[l], CHANS[l + 1]) for l in range(4))
        self.scratch = torch.empty(need, dtype=torch.float32, device=device)
        self.mse_scratch = torch.empty(1024, dtype=torch.float64, device=device)
        self.inv_den = torch.empty(1, dtype=torch.float32, device=device)
        self.loss_dev = torch.empty(1, dtype=torch.float64, device=device)

    def _ensure(self, x0):
        B, H, W, _ = x0.shape
        if (B, H, W) != (self.B, self.H, self.W):
            self._alloc(B, H, W, x0.device)

    def forward(self, x0):
        """x0: (B, H, W, 16) bf16. Returns the (B, H, W, 16) fp32 output buffer."""
        self._ensure(x0)
        self.a[0].copy_(x0)
        for l in range(4):
            last = l == 3
            R.nn_conv_forward(self.a[l], self.wbf[l], self.b32[l], self.y[l], None if last else self.a[l + 1], None,
                              DILS[l], R.NN_EPI_NONE if last else R.NN_EPI_SILU)
        return self.y[3]

    def loss_and_grads(self, x0, tgt, wgt):
        """Forward, weighted MSE against tgt (B, H, W, 3) and backward into gw / gb; returns the loss."""
        out = self.forward(x0)
        R.nn_masked_mse(out, tgt, wgt, self.g[3], self.mse_scratch, self.inv_den, self.loss_dev)
        for l in range(3, -1, -1):
            R.nn_conv_backward_weight(self.a[l], self.g[l], DILS[l], self.gw[l], self.gb[l], self.scratch)
            if l > 0:
                R.nn_flip_weights(self.wbf[l], self.wt[l])
                # g_{l-1} = (dL/da_l) * silu'(y_{l-1})
                R.nn_conv_forward(self.g[l], self.wt[l], None, None, self.g[l - 1], self.y[l - 1], DILS[l],
                                  R.NN_EPI_SILU_GRAD)
        return float(self.loss_dev.item())

    def adam(self, lr):
        self.t += 1
        for l in range(4):
            R.nn_adam(self.w32[l], self.wbf[l], self.gw[l], self.mw[l], self.vw[l], lr, self.t)
            R.nn_adam(self.b32[l], None, self.gb[l], self.mb[l], self.vb[l], lr, self.t)


# ---------------------------------------------------------------------------
# Lattice side: batches of obstacle channels (rD2Q9, walls on the y faces)
# ---------------------------------------------------------------------------

def channel_params(geom, storage="f32dev"):
    return R.make_params(lattice="Q9", equation="NSE", storage=storage, pattern="AA", n=geom["n"], dx=geom["dx"],
                         nu=geom["nu"], force=geom["force"], wall_faces=R.WALL_YM | R.WALL_YP, rho0=1.0)


def make_batch(geoms, storage="f32dev"):
    return R.Batch([channel_params(g, storage) for g in geoms], solids=[g["solid"].astype(np.uint8) for g in geoms])


def cold_start(batch, k):
    """Re-initialise domain k of a batch at rest (rho = 1, u = 0)."""
    d = batch.domains[k]
    d.set_fields(torch.ones(d.N, dtype=torch.float64, device="cuda"),
                 torch.zeros((d.d, d.N), dtype=torch.float64, device="cuda"))


def run_to_steady(batch, tol=1e-6, check=50, max_steps=400_000, log=None, label="", fallback=False,
                  stall_checks=200):
    """Step every domain until its residual (checked every `check` steps, as
    ||u^n - u^(n-check)|| / ||u^n||) falls below tol.

    With fallback=True a domain that was started from a prediction restarts
    cold (rho = 1, u = 0) once, when its residual is not finite or has made no
    new minimum for `stall_checks` consecutive checks; its step count includes
    the steps spent before the restart.  The window must span several sound
    periods of the channel: a start from a predicted field excites sound waves
    that keep the residual from setting a new minimum for a while (the default
    200 checks of 50 steps are over five periods across 512 nodes; 40 checks
    restarted 9 of 16 good warm starts).  Without fallback a non-finite
    residual raises FloatingPointError.

    Returns the step count at convergence per domain (the last step count where
    not converged), the converged flags, the wall time, the total steps, and the
    number of cold restarts per domain."""
    nd = len(batch.domains)
    steps = np.full(nd, -1, dtype=np.int64)
    restarts = np.zeros(nd, dtype=np.int64)
    best = np.full(nd, np.inf)
    since_best = np.zeros(nd, dtype=np.int64)
    batch.residuals()                       # stores the initial velocity
    n = 0
    t0 = time.perf_counter()
    last_log = t0
    while n < max_steps and (steps < 0).any():
        batch.step(check)
        n += check
        r = np.array(batch.residuals())
        bad = ~np.isfinite(r)
        if bad.any() and not fallback:
            raise FloatingPointError(f"non-finite residual in domains {np.where(bad)[0].tolist()}")
        newly = (steps < 0) & ~bad & (r < tol)
        steps[newly] = n
        improved = ~bad & (r < best)
        best[improved] = r[improved]
        since_best[improved] = 0
        since_best[~improved] += 1
        if fallback:
            # a first residual after a (re)start is +inf: it neither improves nor stalls
            stalled = (steps < 0) & (restarts == 0) & (bad | (since_best >= stall_checks))
            for k in np.where(stalled)[0]:
                cold_start(batch, int(k))
                restarts[k] += 1
                best[k] = np.inf
                since_best[k] = 0
            if stalled.any():
                batch.residuals()           # the restarted domains store their new velocity
                if log:
                    log(f"{label} step {n}: cold restart of domains {np.where(stalled)[0].tolist()}")
        if log and time.perf_counter() - last_log > 20.0:
            last_log = time.perf_counter()
            fin = r[np.isfinite(r)]
            log(f"{label} step {n}: {int((steps >= 0).sum())}/{nd} converged, "
                f"max r = {fin.max() if fin.size else float('nan'):.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    conv = steps >= 0
    steps[~conv] = n
    return steps, conv, wall, n, restarts


def geometry_tensors(geoms, device="cuda"):
    solid = torch.tensor(np.stack([g["solid"].reshape(g["n"][1], g["n"][0]) for g in geoms]).astype(np.uint8),
                         device=device)
    re = torch.tensor(np.array([g["Re"] for g in geoms], dtype=np.float32), device=device)
    return solid, re


def features(geoms, device="cuda"):
    g0 = geoms[0]
    nx, ny = g0["n"][0], g0["n"][1]
    B = len(geoms)
    solid, re = geometry_tensors(geoms, device)
    x0 = torch.empty((B, ny // COARSEN, nx // COARSEN, CHANS[0]), dtype=torch.bfloat16, device=device)
    R.nn_features(solid, re, B, nx, ny, COARSEN, g0["dx"][1], RE_SCALE, x0)
    return x0, solid


def steady_targets(batch, geoms, device="cuda"):
    """Coarse training targets and weights from the converged fields of a batch."""
    g0 = geoms[0]
    nx, ny = g0["n"][0], g0["n"][1]
    N = nx * ny
    B = len(geoms)
    rho = torch.empty((B, N), dtype=torch.float64, device=device)
    u = torch.empty((B, 2, N), dtype=torch.float64, device=device)
    for k, d in enumerate(batch.domains):
        r_k, u_k = d.moments()
        rho[k].copy_(r_k)
        u[k].copy_(u_k)
    solid, _ = geometry_tensors(geoms, device)
    tgt = torch.empty((B, ny // COARSEN, nx // COARSEN, 3), dtype=torch.float32, device=device)
    wgt = torch.empty((B, ny // COARSEN, nx // COARSEN), dtype=torch.float32, device=device)
    R.nn_targets(rho, u, solid, B, nx, ny, COARSEN, g0["dx"][1], g0["Ut"], RHO_SCALE, tgt, wgt)
    return tgt, wgt


def initial_fields(geoms, out=None, device="cuda"):
    """rho, u on the nodes from a network output (None: the Poiseuille prior alone)."""
    g0 = geoms[0]
    nx, ny = g0["n"][0], g0["n"][1]
    B = len(geoms)
    if out is None:
        out = torch.zeros((B, ny // COARSEN, nx // COARSEN, CHANS[-1]), dtype=torch.float32, device=device)
    solid, _ = geometry_tensors(geoms, device)
    rho = torch.empty((B, nx * ny), dtype=torch.float64, device=device)
    u = torch.empty((B, 2, nx * ny), dtype=torch.float64, device=device)
    R.nn_warm_fields(out, B, nx, ny, COARSEN, g0["dx"][1], g0["Ut"], RHO_SCALE, solid, rho, u)
    return rho, u


def apply_initial(batch, rho, u):
    for k, d in enumerate(batch.domains):
        d.set_fields(rho[k], u[k], with_fne=True)


def train(net, X, T, Wt, epochs, batch_size, lr, seed=0, log=None):
    """Minibatch Adam over (X, T, Wt) device tensors; returns the loss history per epoch."""
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    hist = []
    for ep in range(epochs):
        perm = rng.permutation(n)
        tot, cnt = 0.0, 0
        for s in range(0, n - batch_size + 1, batch_size):
            idx = torch.tensor(perm[s:s + batch_size], device=X.device)
            loss = net.loss_and_grads(X[idx].contiguous(), T[idx].contiguous(), Wt[idx].contiguous())
            net.adam(lr * (0.5 * (1 + math.cos(math.pi * ep / max(1, epochs)))))
            tot += loss
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log(f"epoch {ep}: mean loss {hist[-1]:.4e}")
    return hist


def predict(net, geoms, chunk=16):
    x0, _ = features(geoms)
    outs = []
    for s in range(0, x0.shape[0], chunk):
        outs.append(net.forward(x0[s:s + chunk].contiguous()).clone())
    return torch.cat(outs, 0), x0
