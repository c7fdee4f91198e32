"""FP64 offset min-sum (OMS) with learned offsets: forward pass, training loss
and gradients. CPU oracle for the differentiable decoder.

TEST INFRASTRUCTURE, under the same rules as the rest of this package: only the
test suite, the smoke check and the benchmark's CPU-baseline leg may use it,
and it shares no code with the product library. Plain PyTorch CPU operations in
float64; the gradients are torch autograd's.

What it computes (the decoder the integer path approximates, with the check
node simplified to offset min-sum, the simplification the paper cites as the
usual alternative to full BP, Sec. 2; the offsets are per iteration and per
base-matrix edge):

* State: soft values E_j (init: the channel LLRs) and CN->VN messages L_e
  (init 0), updated by the layered schedule of Sec. 2: layers in ascending
  order, and within a layer every row at once (the rows of a QC layer touch
  distinct columns).
* Row i of layer b with edges k to columns j_k: v_k = E_{j_k} - L_k (Eq. 8);
  sigma_k = (-1)^{s_i} * prod_{k'} sgn(v_{k'}) * sgn(v_k) with sgn(0) = +1
  (syndrome decoding); L_k = sigma_k * max(min_{k' != k} |v_{k'}| - beta_{t,e(k)}, 0);
  E_{j_k} = v_k + L_k (Eq. 9, no saturation in floating point). Ties between
  minima go to the lowest edge index (the paper does not address ties; the
  choice only decides which tied input the gradient reaches).
* T iterations, no early stop. Loss of a frame:
  sum_t w_t * sum_j softplus(-(1 - 2 x_j) * E_j^(t)) / n, with E^(t) the soft
  values after iteration t and x the transmitted word (binary cross-entropy of
  the bit decisions).
"""
from __future__ import annotations

import numpy as np
import torch


def _layers(base):
    """Per layer: the base columns with a circulant, their shifts and block
    indices (blocks numbered row-major over the base matrix)."""
    base = np.asarray(base)
    out, blk = [], 0
    for b in range(base.shape[0]):
        cols, shifts, blks = [], [], []
        for c in range(base.shape[1]):
            if base[b, c] >= 0:
                cols.append(c)
                shifts.append(int(base[b, c]))
                blks.append(blk)
                blk += 1
        out.append((cols, shifts, blks))
    return out, blk


def _first_min(a, ks, d):
    """[F, 1, Z] index of the first minimum over dim 1 (no gradient)."""
    with torch.no_grad():
        lo = a.min(dim=1, keepdim=True).values
        return torch.where(a == lo, ks, d).min(dim=1, keepdim=True).values


def unpack_syndrome(syn_packed, m):
    """uint8 [F, ceil(m/8)] LSB-first -> int [F, m]."""
    return np.unpackbits(np.asarray(syn_packed, dtype=np.uint8), axis=-1, bitorder="little")[..., :m].astype(np.int64)


def oms_forward(base, z: int, syn_bits, llr, beta, x_bits, weights=None):
    """Returns (loss [F], E_final [F, n], E_iter [T, F, n]) as float64 tensors.
    syn_bits: [F, m] 0/1; llr: [F, n]; beta: [T, n_blocks] (may require grad);
    x_bits: [F, n] 0/1; weights: [T] or None (all ones)."""
    layers, nblk = _layers(base)
    base = np.asarray(base)
    mb, nb = base.shape
    llr = torch.as_tensor(llr, dtype=torch.float64)
    beta = torch.as_tensor(beta, dtype=torch.float64)
    T = beta.shape[0]
    if beta.shape[1] != nblk:
        raise ValueError("beta must be [T, n_blocks]")
    F = llr.shape[0]
    w = torch.ones(T, dtype=torch.float64) if weights is None else torch.as_tensor(weights, dtype=torch.float64)
    syn = torch.as_tensor(np.asarray(syn_bits), dtype=torch.float64).reshape(F, mb, z)
    ysign = 1.0 - 2.0 * torch.as_tensor(np.asarray(x_bits), dtype=torch.float64)
    n = nb * z
    # E per base column, [F, Z]; row r of a block with shift s reads column entry (r + s) mod Z
    E = [llr[:, c * z:(c + 1) * z] for c in range(nb)]
    L = {}
    for b, (cols, shifts, blks) in enumerate(layers):
        for k in range(len(cols)):
            L[(b, k)] = torch.zeros(F, z, dtype=torch.float64)
    E_iter = []
    loss = torch.zeros(F, dtype=torch.float64)
    for t in range(T):
        for b, (cols, shifts, blks) in enumerate(layers):
            d = len(cols)
            v = torch.stack([torch.roll(E[c], -s, dims=1) - L[(b, k)]
                             for k, (c, s) in enumerate(zip(cols, shifts))], dim=1)   # [F, d, Z]
            sg = torch.where(v < 0, -1.0, 1.0).to(torch.float64)
            total = (1.0 - 2.0 * syn[:, b, :]) * torch.prod(sg, dim=1)                 # [F, Z]
            sigma = total[:, None, :] * sg
            a = v.abs()
            # minimum and second minimum; ties go to the lowest edge index
            ks = torch.arange(d)[None, :, None]
            i1 = _first_min(a, ks, d)
            m1 = a.gather(1, i1)
            masked = a.scatter(1, i1, float("inf"))
            i2 = _first_min(masked, ks, d)
            m2 = masked.gather(1, i2)
            mex = torch.where(ks == i1, m2, m1)
            off = beta[t, blks][None, :, None]
            lnew = sigma * torch.relu(mex - off)
            for k, (c, s) in enumerate(zip(cols, shifts)):
                L[(b, k)] = lnew[:, k, :]
                E[c] = torch.roll(v[:, k, :] + lnew[:, k, :], s, dims=1)
        Et = torch.cat(E, dim=1)
        E_iter.append(Et)
        loss = loss + w[t] * torch.nn.functional.softplus(-ysign * Et).sum(dim=1) / n
    return loss, E_iter[-1] if E_iter else llr, torch.stack(E_iter) if E_iter else llr[None]


def oms_grad(base, z: int, syn_bits, llr, beta, x_bits, weights=None, dloss=None):
    """Gradients of sum_f dloss_f * loss_f (dloss = ones by default) with
    respect to beta [T, n_blocks] and the channel LLRs [F, n]; also the loss."""
    beta = torch.tensor(np.asarray(beta, dtype=np.float64), requires_grad=True)
    llr = torch.tensor(np.asarray(llr, dtype=np.float64), requires_grad=True)
    loss, _, _ = oms_forward(base, z, syn_bits, llr, beta, x_bits, weights)
    g = torch.ones_like(loss) if dloss is None else torch.as_tensor(dloss, dtype=torch.float64)
    db, dl = torch.autograd.grad((loss * g).sum(), [beta, llr], allow_unused=True)
    if dl is None:
        dl = torch.zeros_like(llr)
    return {"loss": loss.detach().numpy(), "dbeta": db.numpy(), "dllr": dl.numpy()}
