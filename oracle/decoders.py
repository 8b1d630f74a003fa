"""MS / SMS / SAGMS / BP decoding on the binary Tanner graph (test oracle).

Follows Section II (BP4 decoder, eqs. (bp4_vn), (bp4_cn); MS and SMS
decoders, eq. (ms_cn)), Section III (syndrome ratio eq. (synratio), adaptive
effective gain eq. (alphaeff), SAGMS update eq. (sagms_cn)) and the control
flow of Algorithm 1, on the binary Tanner graph of one CSS check matrix H
(this project's reading: the X part of the error is decoded from its H_Z
syndrome with the binary prior LLR).

Readings where the paper is silent or inconsistent (each listed in the
design notes of the project):
  * Round order.  Messages start as v2c = L0 on every edge and c2v = 0, so
    the first posterior is L0 and the first hard decision [L0 < 0] (all
    zero for a positive prior); if its residual syndrome is zero the frame
    is done after 0 rounds.  Otherwise each round l = 1..lmax is: gains from
    the current residual syndrome, CN update, VN update, posterior and hard
    decision, residual syndrome s_res = s xor H e_hat, and exit if
    s_res = 0.  `iters` counts the CN updates performed (l at convergence,
    lmax otherwise).  This is Algorithm 1 with its top-of-loop test also
    applied after the lmax-th update, so that every update performed is
    used.
  * The CN sign uses the original syndrome bit s_i (eqs. (ms_cn),
    (sagms_cn)); the residual bit s_res_i only selects the eta boost
    (eq. (alphaeff)).  |S| in the syndrome ratio is m, the number of rows
    of H (redundant rows included).
  * sgn(x) = -1 iff x < 0, so both signed zeros count as positive; the
    hard decision is e_hat_j = [posterior_j < 0] (the binary reading of the
    argmin over Paulis in Algorithm 1).
  * The SAGMS gain of eq. (alphaeff) is g = a_max - (a_max - a_min) * w/m
    with w = ||s_res||_0, times eta at unsatisfied checks; it is computed
    in IEEE double from (a_min, a_max, eta).
  * BP: the phi-form sum is floored at -ln(1 - 2^-40), capping the output
    magnitude at 2 atanh(1 - 2^-40) ~ 28.42, so that a check whose other
    inputs are all very reliable does not emit an infinite message.

Arithmetic modes
  "fp64"  definitional: the CN output of every edge is computed from its
          own exclusion set (no min1/min2 shortcut), the VN message of every
          edge is L0 + the sum over the other checks (eq. (bp4_vn)), all
          in IEEE double.  Gains in double.
  "fp32"  the same steps with FP32 messages, in the one operation order
          a device implementation can reproduce bit for bit:
            gain       = float32(double gain above)
            CN output  = sign * float32(gain * exclusive min)  (exact min)
            posterior  = ((L0 + c_1) + c_2) + ... over the variable's
                         checks in ascending check index, FP32 adds
            VN message = float32(posterior - own c2v)
          BP in this mode evaluates the CN in double from FP32 inputs and
          rounds the output to FP32.
  "fp16"  reduced-precision messages with FP32 posteriors: every v2c and
          c2v message is saturated to the largest finite half (+-65504) and
          rounded to IEEE half (round to nearest even):
            v2c       = half(posterior - c2v)       (FP32 difference)
            CN output = sign * half(float32(gain) * exclusive min)
            posterior = FP32 sum as in "fp32" (the first v2c is half(L0))
          The prior is first put on the grid of step 2^-24 (values of
          magnitude >= 1 are already on it): every half is a multiple of
          2^-24, so every posterior and v2c is one too, and a v2c is either
          +0 or at least 2^-24 in magnitude -- it never rounds to -0, and its
          sign (sgn(0) = +1) is the sign of the unrounded FP32 difference.
  "int6"  6-bit magnitude plus sign on a grid of step 1/4 (range +-15.75):
          q(x) = clip(round_half_even(4 x), -63, 63) / 4; the prior is
          quantized too, L0' = q(L0), so posteriors L0' + sum c2v are exact
            v2c       = q(posterior - c2v)          (saturating)
            CN output = sign * q(float32(gain) * exclusive min)
  The two quantized modes apply to the min-sum family only.
  Signed zeros of L0 are read as +0 in all modes.
  The order of a variable's checks in the FP32 posterior sum is part of the
  graph: ascending check index by default, or an explicit order (for a GB
  code, the order of the terms of its polynomials; codes.gb_var_checks).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

KINDS = ("ms", "sms", "sagms", "bp")
ARITH = ("fp64", "fp32", "fp16", "int6")


def grid24(x):
    """x rounded to a multiple of 2^-24 (nearest even), -0 read as +0."""
    x = np.asarray(x, dtype=np.float32)
    small = np.abs(x) < 1.0
    r = np.where(small, np.rint(x * np.float32(2.0 ** 24)) * np.float32(2.0 ** -24), x).astype(np.float32)
    return r + np.float32(0.0)


def quantize(x, arith):
    """The message rounding of a reduced-precision mode (identity otherwise)."""
    x = np.asarray(x, dtype=np.float32)
    if arith == "fp16":
        return np.clip(x, -65504.0, 65504.0).astype(np.float16).astype(np.float32)
    if arith == "int6":
        return (np.clip(np.rint(x * np.float32(4.0)), -63.0, 63.0) * np.float32(0.25)).astype(np.float32)
    return x
# phi-form floor used by the BP check update (see module notes)
BP_PHI_FLOOR = -np.log1p(-(2.0 ** -40))


@dataclass
class DecoderParams:
    kind: str = "sagms"
    lmax: int = 100
    alpha: float = 0.75          # SMS scale
    alpha_min: float = 0.30      # SAGMS (Section V setup values)
    alpha_max: float = 0.50
    eta: float = 1.10

    def validate(self):
        if self.kind not in KINDS:
            raise ValueError("unknown decoder kind %r" % self.kind)
        if self.lmax < 1:
            raise ValueError("lmax must be >= 1")
        if self.kind == "sms" and not (0.0 < self.alpha <= 1.0):
            raise ValueError("SMS alpha must lie in (0, 1]")
        if self.kind == "sagms":
            if not (0.0 < self.alpha_min <= 1.0 and 0.0 < self.alpha_max <= 1.0):
                raise ValueError("alpha_min, alpha_max must lie in (0, 1]")
            if self.eta < 1.0:
                raise ValueError("eta must be >= 1")
            # stability constraint alpha_max * eta <= 1 (Section III)
            if self.alpha_max * self.eta > 1.0:
                raise ValueError("alpha_max * eta must be <= 1")


class TannerGraph:
    """Edge tables of the Tanner graph of a dense 0/1 check matrix H (m x n).

    Edges are numbered check-major (check i's edges are consecutive, in
    ascending variable index).  cn_edge[i] lists check i's edges, vn_edge[j]
    variable j's edges in ascending check index, or in the order given by
    var_checks[j] (a permutation of j's checks); both tables are padded with
    the sentinel index E (one extra message slot).
    """

    def __init__(self, h, var_checks=None):
        h = (np.asarray(h, dtype=np.uint8) & 1)
        self.h = h
        self.m, self.n = h.shape
        rows, cols = np.nonzero(h)          # row-major: check-major order
        self.E = rows.size
        self.e_check = rows.astype(np.int64)
        self.e_var = cols.astype(np.int64)
        self.cn_deg = h.sum(axis=1).astype(np.int64)
        self.vn_deg = h.sum(axis=0).astype(np.int64)
        if (self.cn_deg == 1).any():
            raise ValueError("checks of degree 1 are not supported")
        self.dc = int(self.cn_deg.max()) if self.m else 0
        self.dv = int(self.vn_deg.max()) if self.n else 0
        self.cn_edge = np.full((self.m, max(self.dc, 1)), self.E, dtype=np.int64)
        self.vn_edge = np.full((self.n, max(self.dv, 1)), self.E, dtype=np.int64)
        fill_c = np.zeros(self.m, dtype=np.int64)
        fill_v = np.zeros(self.n, dtype=np.int64)
        for e in range(self.E):            # edges arrive in ascending (i, j)
            i, j = self.e_check[e], self.e_var[e]
            self.cn_edge[i, fill_c[i]] = e
            fill_c[i] += 1
            self.vn_edge[j, fill_v[j]] = e  # ascending check index
            fill_v[j] += 1
        if var_checks is not None:
            edge_of = {(int(self.e_check[e]), int(self.e_var[e])): e for e in range(self.E)}
            for j in range(self.n):
                order = [int(c) for c in var_checks[j]]
                if sorted(order) != sorted(int(self.e_check[e]) for e in self.vn_edge[j] if e < self.E):
                    raise ValueError("var_checks[%d] is not a permutation of the variable's checks" % j)
                self.vn_edge[j, :len(order)] = [edge_of[(c, j)] for c in order]


def check_gains(p: DecoderParams, sres: np.ndarray, m: int) -> np.ndarray:
    """Per-check gain alpha_i in double, [F, m] (eq. (alphaeff) for SAGMS)."""
    f = sres.shape[0]
    if p.kind in ("ms", "bp"):
        return np.ones((f, m))
    if p.kind == "sms":
        return np.full((f, m), float(p.alpha))
    w = sres.sum(axis=1).astype(np.float64)            # ||s_res||_0
    gamma = w / float(m)                                 # eq. (synratio), |S| = m
    g = p.alpha_max - (p.alpha_max - p.alpha_min) * gamma
    return np.where(sres.astype(bool), (g * p.eta)[:, None], g[:, None])


def _neg(x):
    return x < 0


def cn_minsum(v: np.ndarray, s: np.ndarray, gain: np.ndarray, arith: str = "fp64") -> np.ndarray:
    """Eq. (ms_cn) / (sagms_cn) for every check position, by exclusion.

    v [F, m, d] incoming VN->CN messages (padding slots hold +inf),
    s [F, m] original syndrome bits, gain [F, m].  Returns [F, m, d]:
      out[p] = (-1)^s * prod_{q != p} sgn(v[q]) * gain * min_{q != p} |v[q]|.
    The product gain * min is rounded in the dtype of `v`, then to the
    message format of `arith` ("fp16", "int6").
    """
    d = v.shape[-1]
    other = ~np.eye(d, dtype=bool)                       # [p, q]: q != p
    mag = np.abs(v)
    excl_min = np.where(other, mag[..., None, :], np.inf).min(axis=-1)
    neg = _neg(v)
    par = ((neg[..., None, :] & other).sum(axis=-1) + s[..., None]) & 1
    out = gain.astype(v.dtype)[..., None] * excl_min
    if arith in ("fp16", "int6"):
        out = quantize(out, arith)
    return np.where(par.astype(bool), -out, out)


def _phi(x):
    # Gallager phi(x) = -ln tanh(x/2); phi(0) = +inf, phi(+inf) = 0
    with np.errstate(divide="ignore"):
        return -np.log(np.tanh(x / 2.0))


def cn_bp(v: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Eq. (bp4_cn) in the phi form, by exclusion, evaluated in double.

    out[p] = (-1)^s prod_{q != p} sgn(v[q]) * phi( sum_{q != p} phi(|v[q]|) ),
    with the phi-sum floored at BP_PHI_FLOOR.  Padding slots (+inf) give
    phi = 0 and leave the sum unchanged.  Output in the dtype of `v`.
    """
    d = v.shape[-1]
    other = ~np.eye(d, dtype=bool)
    mag = np.abs(v.astype(np.float64))
    ph = _phi(mag)
    ssum = np.where(other, ph[..., None, :], 0.0).sum(axis=-1)
    ssum = np.maximum(ssum, BP_PHI_FLOOR)
    outmag = _phi(ssum)
    neg = _neg(v)
    par = ((neg[..., None, :] & other).sum(axis=-1) + s[..., None]) & 1
    out = np.where(par.astype(bool), -outmag, outmag)
    return out.astype(v.dtype)


@dataclass
class DecodeResult:
    ehat: np.ndarray        # [F, n] uint8
    iters: np.ndarray       # [F] int32
    converged: np.ndarray   # [F] bool
    posterior: np.ndarray   # [F, n] last posterior of every frame
    trace: list | None = None


def decode(g: TannerGraph, synd, llr0, params: DecoderParams, arith: str = "fp64",
           early_exit: bool = True, trace: bool = False, chunk: int = 1024) -> DecodeResult:
    """Decode a batch of syndromes (Algorithm 1 with the readings above).

    synd [F, m] 0/1, llr0 [n] prior LLRs.  With early_exit=False every frame
    runs exactly lmax rounds (used by the tree-graph pins).  With trace=True
    the messages of every round are recorded (small batches only).
    """
    params.validate()
    synd = np.asarray(synd, dtype=np.uint8) & 1
    f = synd.shape[0]
    if f > chunk and not trace:
        parts = [decode(g, synd[a:a + chunk], llr0, params, arith, early_exit, False, chunk)
                 for a in range(0, f, chunk)]
        return DecodeResult(np.concatenate([r.ehat for r in parts]),
                            np.concatenate([r.iters for r in parts]),
                            np.concatenate([r.converged for r in parts]),
                            np.concatenate([r.posterior for r in parts]))
    if arith not in ARITH:
        raise ValueError("arith must be one of %s" % (ARITH,))
    if arith in ("fp16", "int6") and params.kind == "bp":
        raise ValueError("reduced-precision messages apply to the min-sum family only")
    dt = np.float64 if arith == "fp64" else np.float32
    m, n, E = g.m, g.n, g.E
    L0 = np.asarray(llr0, dtype=np.float64).astype(dt) + dt(0.0)   # -0 -> +0
    if arith == "int6":
        L0 = quantize(L0, arith) + dt(0.0)                          # a prior rounding to -0 reads as +0
    if arith == "fp16":
        L0 = grid24(L0)
    if L0.shape != (n,):
        raise ValueError("llr0 must have n entries")

    # round 0: posterior L0, hard decision [L0 < 0], its residual syndrome
    e0 = (L0 < 0).astype(np.uint8)
    ehat = np.broadcast_to(e0, (f, n)).copy()
    iters = np.zeros(f, dtype=np.int32)
    conv = np.zeros(f, dtype=bool)
    post_all = np.broadcast_to(L0, (f, n)).copy()
    sres = synd ^ ((g.h.astype(np.int64) @ e0.astype(np.int64)) & 1).astype(np.uint8)[None, :]
    active = sres.any(axis=1) if early_exit else np.ones(f, dtype=bool)
    conv[~sres.any(axis=1)] = True

    # message slots: E edges plus the padding sentinel
    v2c = np.empty((f, E + 1), dtype=dt)
    v2c[:, :E] = quantize(L0[g.e_var], arith) if arith in ("fp16", "int6") else L0[g.e_var]
    v2c[:, E] = np.inf
    c2v = np.zeros((f, E + 1), dtype=dt)
    vn_valid = g.vn_edge < E
    rounds = []

    for ell in range(1, params.lmax + 1):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        s_i = synd[idx]
        # (i) gains from the current residual syndrome
        gain = check_gains(params, sres[idx], m)
        # (ii) CN update on every check
        vin = v2c[idx][:, g.cn_edge]                      # [F', m, dc]
        if params.kind == "bp":
            cout = cn_bp(vin, s_i)
        else:
            cout = cn_minsum(vin, s_i, gain, arith)
        cnew = np.zeros((idx.size, E + 1), dtype=dt)
        valid_c = g.cn_edge < E
        cnew[:, g.cn_edge[valid_c]] = cout[:, valid_c]
        # (iii) VN update and posterior
        cj = cnew[:, g.vn_edge]                           # [F', n, dv], pad -> 0
        vnew = np.empty((idx.size, E + 1), dtype=dt)
        vnew[:, E] = np.inf
        if arith == "fp64":
            other = ~np.eye(g.vn_edge.shape[1], dtype=bool)
            excl = np.where(other & vn_valid[:, None, :], cj[:, :, None, :], 0.0).sum(axis=-1)
            vmsg = L0[None, :, None] + excl                   # [F', n, dv]
            vnew[:, g.vn_edge[vn_valid]] = vmsg[:, vn_valid]
            post = L0[None, :] + np.where(vn_valid, cj, 0.0).sum(axis=-1)
        else:
            post = np.broadcast_to(L0, (idx.size, n)).copy()
            for r in range(g.vn_edge.shape[1]):               # ascending check order
                post = np.where(vn_valid[None, :, r], post + cj[:, :, r], post)
            vnew[:, :E] = post[:, g.e_var] - cnew[:, :E]
            if arith in ("fp16", "int6"):
                vnew[:, :E] = quantize(vnew[:, :E], arith)
        # (iv) hard decision and (v) residual syndrome
        e = (post < 0).astype(np.uint8)
        r_new = s_i ^ (((e.astype(np.int64) @ g.h.T.astype(np.int64)) & 1).astype(np.uint8))
        c2v[idx] = cnew
        v2c[idx] = vnew
        ehat[idx] = e
        sres[idx] = r_new
        post_all[idx] = post
        iters[idx] = ell
        done = ~r_new.any(axis=1)
        if early_exit:
            conv[idx[done]] = True
            active[idx[done]] = False
        else:
            conv[idx] = done
        if trace:
            rounds.append(dict(frames=idx.copy(), c2v=cnew[:, :E].copy(), v2c=vnew[:, :E].copy(),
                               post=post.copy(), gain=gain.copy(), sres=r_new.copy()))
    return DecodeResult(ehat, iters, conv, post_all, rounds if trace else None)
