"""Layered (check-serial) schedule for the min-sum family (test oracle).

The paper runs Algorithm 1 with the flooding schedule: every check node
updates from the previous round's variable messages, then every variable.
This module is the layered alternative that the design notes list beside
it.  The paper defines no layered schedule, so everything here is this
project's reading (each point is listed in the design notes):

  * Layers.  The checks are split into layers of checks with pairwise
    disjoint supports by first fit in ascending check index: check i joins
    the first layer none of whose checks shares a variable with it, or
    opens a new layer.  Layers run in the order they were opened; within a
    layer the order does not matter (disjoint supports), so a whole layer
    may be updated at once.
  * Round.  One round visits every layer once.  For each check i of the
    layer and each variable j of check i: v2c = post_j - c2v_old(i->j);
    the check output c2v_new(i->j) follows eq. (ms_cn) / (sagms_cn) from
    these v2c values, exactly as in the flooding schedule; then
    post_j = v2c + c2v_new(i->j).  So later layers of a round already see
    the messages of earlier layers (the schedule's point).
  * Gains.  The SAGMS gains of a round come from the residual syndrome at
    the start of the round (eqs. (synratio), (alphaeff)), as in flooding;
    the eta boost is selected by the residual bit of the updated check.
  * Rounds, hard decisions, exit test and what l_max counts are those of
    the flooding decoder: start with post = L0 and c2v = 0, test the
    hard decision [L0 < 0] first (0 rounds), then after every round.

Arithmetic modes
  "fp64"  definitional: v2c(j->i) = L0_j + sum over the other checks k of j
          of the current c2v(k->j), and the posterior recomputed as L0_j +
          the sum of all current c2v into j, in IEEE double.
  "fp32"  the incremental order a device implementation uses, in FP32:
          v2c = fl(post - c2v_old), post = fl(v2c + c2v_new).
BP is not offered with this schedule.
"""
from __future__ import annotations

import numpy as np

from .decoders import DecodeResult, DecoderParams, TannerGraph, check_gains, cn_minsum


def greedy_layers(h) -> list[np.ndarray]:
    """First-fit partition of the checks of h into layers of checks with
    pairwise disjoint supports, scanning checks in ascending index."""
    h = np.asarray(h, dtype=np.uint8) & 1
    layers: list[list[int]] = []
    used: list[np.ndarray] = []
    for i in range(h.shape[0]):
        row = h[i].astype(bool)
        for t in range(len(layers)):
            if not (used[t] & row).any():
                layers[t].append(i)
                used[t] |= row
                break
        else:
            layers.append([i])
            used.append(row.copy())
    return [np.asarray(x, dtype=np.int64) for x in layers]


def decode_layered(g: TannerGraph, synd, llr0, params: DecoderParams, arith: str = "fp64",
                   layers=None, chunk: int = 1024) -> DecodeResult:
    """Decode a batch of syndromes with the layered schedule (module notes)."""
    params.validate()
    if params.kind == "bp":
        raise ValueError("the layered schedule covers the min-sum family only")
    if arith not in ("fp64", "fp32"):
        raise ValueError("the layered schedule has fp64 and fp32 modes")
    synd = np.asarray(synd, dtype=np.uint8) & 1
    f = synd.shape[0]
    if layers is None:
        layers = greedy_layers(g.h)
    if f > chunk:
        parts = [decode_layered(g, synd[a:a + chunk], llr0, params, arith, layers, chunk)
                 for a in range(0, f, chunk)]
        return DecodeResult(np.concatenate([r.ehat for r in parts]), np.concatenate([r.iters for r in parts]),
                            np.concatenate([r.converged for r in parts]),
                            np.concatenate([r.posterior for r in parts]))
    dt = np.float64 if arith == "fp64" else np.float32
    m, n, E = g.m, g.n, g.E
    L0 = np.asarray(llr0, dtype=np.float64).astype(dt) + dt(0.0)   # -0 -> +0
    if L0.shape != (n,):
        raise ValueError("llr0 must have n entries")
    hT = g.h.T.astype(np.int64)

    e0 = (L0 < 0).astype(np.uint8)
    ehat = np.broadcast_to(e0, (f, n)).copy()
    iters = np.zeros(f, dtype=np.int32)
    sres = synd ^ ((e0.astype(np.int64) @ hT) & 1).astype(np.uint8)[None, :]
    conv = ~sres.any(axis=1)
    active = ~conv
    post = np.broadcast_to(L0, (f, n)).copy()
    c2v = np.zeros((f, E + 1), dtype=dt)          # slot E: padding, stays 0
    vn_valid = g.vn_edge < E

    # unscaled min-sum can overflow FP32 on frames that never converge; IEEE
    # infinities and NaNs then take their course (a NaN posterior decides 0)
    with np.errstate(over="ignore", invalid="ignore"):
        return _rounds(g, synd, L0, params, arith, layers, ehat, iters, sres, conv, active, post, c2v, vn_valid, hT)


def _rounds(g, synd, L0, params, arith, layers, ehat, iters, sres, conv, active, post, c2v, vn_valid, hT):
    m, E = g.m, g.E
    dt = L0.dtype.type
    for ell in range(1, params.lmax + 1):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        gain = check_gains(params, sres[idx], m)               # from the round's start
        c = c2v[idx]
        p = post[idx]
        for lay in layers:
            edges = g.cn_edge[lay]                             # [|lay|, dc], padded with E
            valid = edges < E
            var = np.where(valid, g.e_var[np.minimum(edges, E - 1)], 0)
            if arith == "fp64":
                # definitional: L0_j + the current messages of j's other checks
                ve = g.vn_edge[var]                            # [|lay|, dc, dv]
                other = (ve != edges[:, :, None]) & (ve < E)
                v = L0[var][None] + np.where(other[None], c[:, ve], 0.0).sum(axis=-1)
            else:
                v = p[:, var] - c[:, edges]
            v = np.where(valid[None], v, np.inf)
            out = cn_minsum(v, synd[idx][:, lay], gain[:, lay], arith)
            out = np.where(valid[None], out, 0.0).astype(dt)
            cols = edges[valid]
            c[:, cols] = out[:, valid]
            if arith == "fp32":
                p[:, var[valid]] = v[:, valid] + out[:, valid]
        if arith == "fp64":
            cj = c[:, g.vn_edge]
            p = L0[None, :] + np.where(vn_valid[None], cj, 0.0).sum(axis=-1)
        e = (p < 0).astype(np.uint8)
        r_new = synd[idx] ^ (((e.astype(np.int64) @ hT) & 1).astype(np.uint8))
        c2v[idx] = c
        post[idx] = p
        ehat[idx] = e
        sres[idx] = r_new
        iters[idx] = ell
        done = ~r_new.any(axis=1)
        conv[idx[done]] = True
        active[idx[done]] = False
    return DecodeResult(ehat, iters, conv, post)
