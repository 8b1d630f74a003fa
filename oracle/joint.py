"""Joint (quaternary) decoding of X and Z errors with scalar messages (test oracle).

The paper's own decoders (Section II, "BP4 decoder"; Section V setup: the
[[126,28]] GB code with the overcomplete m = 126 check matrix, d_c = d_v = 10)
work on the quaternary Tanner graph: every check row is a Pauli string over
{I, X, Y, Z}, every message is one real number, and each variable keeps
beliefs over all four Paulis.  The Section I footnote names the reduction of
quaternary messages to scalar LLRs it uses: the log-domain scalar-message
BP4 of Lai and Kuo (2021), also used by the overcomplete-check decoders it
cites.  This module restates that decoder from its definitions, with the
check-node rules of eqs. (bp4_cn), (ms_cn) and (sagms_cn), the gains of
eqs. (alphaeff) and (synratio) and the control flow of Algorithm 1.

Definitions (W ranges over the three non-identity Paulis X, Y, Z):
  * Prior.  Lambda_j^W = ln(P(E_j = I) / P(E_j = W)); for the depolarizing
    channel of Section II every W has Lambda^W = L0 = ln((1 - e0) / (e0 / 3)),
    the paper's L0.
  * Posterior beliefs (the VN update, eq. (bp4_vn) in quaternary form).  A
    check message Delta_{i->j} is the log-ratio "E_j commutes with the check's
    Pauli S_ij" over "anticommutes"; it moves every hypothesis W that
    anticommutes with S_ij (on one qubit: W != S_ij):
        Gamma_j^W = Lambda_j^W + sum_{i in M(j), W != S_ij} Delta_{i->j},
    and the extrinsic Gamma_{j->i}^W leaves out check i's own message.
  * Scalarization (VN -> CN message, the footnote's reduction).  With P =
    S_ij, the commuting Paulis are {I, P} and the anticommuting ones the
    other two {A, A'}:
        BP     lambda = ln(1 + e^{-G^P}) - ln(e^{-G^A} + e^{-G^A'})
        MS     lambda = min(G^A, G^A') - min(0, G^P)
    (G = Gamma_{j->i}; the min-sum form is the max-log form of the BP one).
    For a uniform prior L0 > 0 the min-sum message before any check update
    is exactly L0, so Algorithm 1's initialisation "L_{j->i} <- L0" and
    Remark 1's statement that every incoming magnitude of round 1 equals L0
    hold literally for MS, SMS and SAGMS.  For BP the exact form gives
    ln((e^{L0} + 1) / 2) in round 1 (for the depolarizing prior this is the
    binary marginal ln((1 - 2e0/3) / (2e0/3))); this module takes the exact
    form for BP so that BP is exact on trees.
  * CN update: the binary rules on the scalar messages, sign (-1)^{s_i} from
    the original syndrome bit, gain from the residual syndrome (as in the
    binary decoder, decoders.py).
  * Hard decision (Algorithm 1): E_hat_j = argmin over (I, X, Y, Z) of
    (0, Gamma^X, Gamma^Y, Gamma^Z), ties to the first in that order.
  * Residual syndrome (eq. (resid)): s_res_i = s_i xor <S_i, E_hat>, the
    symplectic (trace) inner product; |S| = m in eq. (synratio).

Round order, sgn(0) = +1, gains in IEEE double and the BP phi-sum floor are
those of decoders.py.  One addition: the min-sum family's check outputs
saturate at magnitude MS_CAP = 2^64, |Delta| = min(gain * min|lambda|, 2^64)
(exact in either precision).  Algorithm 1 says nothing about overflow; on
the quaternary graph (d_v = 10) unscaled min-sum magnitudes can grow by up to
(d_v - 1) per round on frames that never converge and would overflow FP32
within lmax = 100 rounds (IEEE infinities, then NaNs from inf - inf in the
scalarization); messages of converging frames stay many orders of magnitude
below the cap.

Arithmetic modes
  "fp64"  definitional: every edge's extrinsic beliefs are the prior plus the
          sum over the variable's other checks; lambda per edge from them.
  "fp32"  FP32 messages in one operation order a device kernel reproduces
          bit for bit (check rows of Paulis X and Z only, i.e. CSS rows):
            S_X, S_Z   = ((D_1 + D_2) + D_3) + ... over the variable's X-type
                         (Z-type) checks in graph order (+0 when there are none)
            Gamma^X    = L0 + S_Z,  Gamma^Z = L0 + S_X,  Gamma^Y = L0 + (S_X + S_Z)
            extrinsic  = Gamma^W - own Delta for the W that the edge moves
            lambda     = (min over the two anticommuting extrinsic values)
                         - min(0, Gamma^P)           (MS family, two roundings)
          and the check update of decoders.py's FP32 mode.  BP in this mode:
          lambda in double from the FP32 beliefs, rounded to FP32.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import gf2
from .decoders import BP_PHI_FLOOR, DecoderParams, check_gains, cn_bp, cn_minsum

# Pauli codes of an edge / a hypothesis: 1 = X, 2 = Y, 3 = Z (0 = I)
PX, PY, PZ = 1, 2, 3
# Saturation of the min-sum family's check outputs (module notes).
MS_CAP = 2.0 ** 64


def pauli_of(sx, sz):
    """Pauli code of symplectic bits (x, z): X = (1, 0), Y = (1, 1), Z = (0, 1)."""
    sx = np.asarray(sx, dtype=np.int64)
    sz = np.asarray(sz, dtype=np.int64)
    return np.where(sx & ~sz & 1, PX, np.where(sx & sz & 1, PY, np.where(sz & 1, PZ, 0)))


def symplectic_syndrome(sx, sz, ex, ez) -> np.ndarray:
    """s_i = <S_i, E> over GF(2): S_x . e_z + S_z . e_x, batched [F, m]."""
    sx = np.asarray(sx, dtype=np.int64)
    sz = np.asarray(sz, dtype=np.int64)
    ex = np.asarray(ex, dtype=np.int64)
    ez = np.asarray(ez, dtype=np.int64)
    return (((ez @ sx.T) + (ex @ sz.T)) & 1).astype(np.uint8)


class PauliGraph:
    """Quaternary Tanner graph of a check matrix of Pauli rows.

    sx, sz [m, n] are the symplectic halves of the rows (X part, Z part).
    Edges are numbered check-major in ascending variable index; e_pauli is
    the Pauli S_ij of each edge.  var_checks[j], if given, lists variable j's
    checks in the order of its FP32 sums (a permutation of its checks;
    default ascending check index).
    """

    def __init__(self, sx, sz, var_checks=None):
        self.sx = np.asarray(sx, dtype=np.uint8) & 1
        self.sz = np.asarray(sz, dtype=np.uint8) & 1
        self.m, self.n = self.sx.shape
        support = (self.sx | self.sz).astype(bool)
        rows, cols = np.nonzero(support)
        self.E = rows.size
        self.e_check = rows.astype(np.int64)
        self.e_var = cols.astype(np.int64)
        self.e_pauli = pauli_of(self.sx[rows, cols], self.sz[rows, cols]).astype(np.int64)
        self.cn_deg = support.sum(axis=1).astype(np.int64)
        self.vn_deg = support.sum(axis=0).astype(np.int64)
        if (self.cn_deg < 2).any():
            raise ValueError("checks of degree < 2 are not supported")
        self.dc = int(self.cn_deg.max())
        self.dv = int(self.vn_deg.max()) if self.n else 0
        self.cn_edge = np.full((self.m, self.dc), self.E, dtype=np.int64)
        self.vn_edge = np.full((self.n, max(self.dv, 1)), self.E, dtype=np.int64)
        fc = np.zeros(self.m, dtype=np.int64)
        fv = np.zeros(self.n, dtype=np.int64)
        for e in range(self.E):
            i, j = self.e_check[e], self.e_var[e]
            self.cn_edge[i, fc[i]] = e
            fc[i] += 1
            self.vn_edge[j, fv[j]] = e
            fv[j] += 1
        if var_checks is not None:
            edge_of = {(int(self.e_check[e]), int(self.e_var[e])): e for e in range(self.E)}
            for j in range(self.n):
                order = [int(c) for c in var_checks[j]]
                mine = sorted(int(self.e_check[e]) for e in self.vn_edge[j] if e < self.E)
                if sorted(order) != mine:
                    raise ValueError("var_checks[%d] is not a permutation of the variable's checks" % j)
                self.vn_edge[j, :len(order)] = [edge_of[(c, j)] for c in order]

    @property
    def css(self) -> bool:
        return not (self.e_pauli == PY).any()


def gb_joint(l: int, a, b):
    """(S_x, S_z, var_checks) of a GB code as one quaternary check matrix.

    Rows 0..l-1 are the X-type checks (rows of H_X = [A | B], Pauli X on
    their support), rows l..2l-1 the Z-type checks (rows of H_Z = [B^T | A^T],
    Pauli Z): m = 2l rows, each of weight |a| + |b|, and every qubit in
    |a| + |b| checks (Section V setup: m = 126, d_c = d_v = 10 for l = 63).
    The FP32 sums take, for variable i < l, the X-type checks (i - a_t) mod l
    and the Z-type checks l + (i + b_t) mod l; for variable l + i the X-type
    checks (i - b_t) mod l and the Z-type checks l + (i + a_t) mod l, each in
    the order of the polynomial terms.
    """
    from .codes import gb_matrices
    hx, hz = gb_matrices(l, a, b)
    n = 2 * l
    sx = np.vstack([hx, np.zeros_like(hz)])
    sz = np.vstack([np.zeros_like(hx), hz])
    vc = []
    for i in range(l):
        vc.append([(i - t) % l for t in a] + [l + (i + t) % l for t in b])
    for i in range(l):
        vc.append([(i - t) % l for t in b] + [l + (i + t) % l for t in a])
    assert len(vc) == n
    return sx, sz, vc


def depolarizing_prior(eps0: float) -> float:
    """The paper's L0 = ln((1 - e0) / (e0 / 3)) (Section II notation)."""
    return float(np.log((1.0 - eps0) / (eps0 / 3.0)))


def _as_prior(llr0, n, dt):
    """[n] (uniform over X, Y, Z) or [n, 3] priors -> [n, 3] in dt, -0 -> +0."""
    p = np.asarray(llr0, dtype=np.float64)
    if p.shape == (n,):
        p = np.repeat(p[:, None], 3, axis=1)
    if p.shape != (n, 3):
        raise ValueError("llr0 must have shape [n] or [n, 3]")
    return p.astype(dt) + dt(0.0)


def hard_decision(gamma) -> tuple[np.ndarray, np.ndarray]:
    """argmin over (I, X, Y, Z) of (0, G^X, G^Y, G^Z), first minimum: (x_hat, z_hat)."""
    g = np.asarray(gamma)
    vals = np.concatenate([np.zeros(g.shape[:-1] + (1,), dtype=g.dtype), g], axis=-1)
    pick = np.argmin(vals, axis=-1)               # numpy argmin: first minimum
    xh = ((pick == PX) | (pick == PY)).astype(np.uint8)
    zh = ((pick == PY) | (pick == PZ)).astype(np.uint8)
    return xh, zh


def scalarize(gext, pauli, kind: str) -> np.ndarray:
    """VN -> CN scalar message from extrinsic beliefs gext [..., 3] (X, Y, Z)
    for edge Paulis `pauli` (broadcast to the leading axes of gext)."""
    g = np.asarray(gext)
    P = np.broadcast_to(np.asarray(pauli), g.shape[:-1])
    gx, gy, gz = g[..., 0], g[..., 1], g[..., 2]
    gp = np.where(P == PX, gx, np.where(P == PY, gy, gz))        # the edge's own Pauli
    ga1 = np.where(P == PX, gy, gx)                              # the two others
    ga2 = np.where(P == PZ, gy, gz)
    if kind == "bp":
        g64 = [x.astype(np.float64) for x in (gp, ga1, ga2)]
        lam = np.logaddexp(0.0, -g64[0]) - np.logaddexp(-g64[1], -g64[2])
        return lam.astype(g.dtype)
    zero = g.dtype.type(0.0)
    return np.minimum(ga1, ga2) - np.minimum(zero, gp)


@dataclass
class JointResult:
    xhat: np.ndarray        # [F, n] uint8, X part of E_hat
    zhat: np.ndarray        # [F, n] uint8, Z part of E_hat
    iters: np.ndarray       # [F] int32
    converged: np.ndarray   # [F] bool
    gamma: np.ndarray       # [F, n, 3] last beliefs (Gamma^X, Gamma^Y, Gamma^Z)
    trace: list | None = None


def _beliefs_fp32(g: PauliGraph, L0, cnew):
    """FP32 posterior beliefs in the order stated in the module notes."""
    f = cnew.shape[0]
    dt = np.float32
    sums = {}
    for typ in (PX, PZ):
        acc = np.zeros((f, g.n), dtype=dt)
        started = np.zeros((f, g.n), dtype=bool)
        for r in range(g.vn_edge.shape[1]):
            e = g.vn_edge[:, r]
            valid = (e < g.E) & (np.where(e < g.E, g.e_pauli[np.minimum(e, g.E - 1)], 0) == typ)
            c = cnew[:, e]                                   # [F, n]
            acc = np.where(valid[None, :], np.where(started, acc + c, c), acc)
            started = started | valid[None, :]
        sums[typ] = acc
    sx, sz = sums[PX], sums[PZ]
    gx = L0[None, :, 0] + sz
    gz = L0[None, :, 2] + sx
    gy = L0[None, :, 1] + (sx + sz)
    return np.stack([gx, gy, gz], axis=-1).astype(dt)


def decode_joint(g: PauliGraph, synd, llr0, params: DecoderParams, arith: str = "fp64",
                 early_exit: bool = True, trace: bool = False, chunk: int = 512) -> JointResult:
    """Joint decode of a batch of syndromes [F, m] (Algorithm 1, module notes).

    llr0: [n] (Lambda^W = llr0[j] for every W) or [n, 3] (X, Y, Z).
    early_exit=False runs every frame for exactly lmax rounds (tree pins).
    """
    params.validate()
    synd = np.asarray(synd, dtype=np.uint8) & 1
    f = synd.shape[0]
    if f > chunk and not trace:
        parts = [decode_joint(g, synd[s:s + chunk], llr0, params, arith, early_exit, False, chunk)
                 for s in range(0, f, chunk)]
        return JointResult(*(np.concatenate([getattr(r, k) for r in parts])
                             for k in ("xhat", "zhat", "iters", "converged", "gamma")))
    if arith not in ("fp64", "fp32"):
        raise ValueError("arith must be fp64 or fp32")
    if arith == "fp32" and not g.css:
        raise ValueError("the FP32 order is defined for rows of Paulis X and Z only")
    dt = np.float64 if arith == "fp64" else np.float32
    m, n, E = g.m, g.n, g.E
    L0 = _as_prior(llr0, n, dt)
    kind = params.kind
    sckind = "bp" if kind == "bp" else "ms"
    moves = (np.arange(1, 4)[None, :] != g.e_pauli[:, None])          # [E, 3]: W anticommutes with S_e

    # round 0: beliefs = prior, its hard decision and residual
    gamma = np.broadcast_to(L0, (f, n, 3)).copy()
    xh, zh = hard_decision(gamma)
    sres = synd ^ symplectic_syndrome(g.sx, g.sz, xh, zh)
    iters = np.zeros(f, dtype=np.int32)
    conv = ~sres.any(axis=1)
    active = ~conv if early_exit else np.ones(f, dtype=bool)

    v2c = np.empty((f, E + 1), dtype=dt)
    v2c[:, :E] = scalarize(L0[g.e_var], g.e_pauli, sckind)[None, :]
    v2c[:, E] = np.inf
    rounds = []
    vn_valid = g.vn_edge < E

    for ell in range(1, params.lmax + 1):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        s_i = synd[idx]
        gain = check_gains(params, sres[idx], m)
        vin = v2c[idx][:, g.cn_edge]
        if kind == "bp":
            cout = cn_bp(vin, s_i)
        else:
            cout = cn_minsum(vin, s_i, gain, arith)
            cout = np.where(cout < 0, -np.minimum(-cout, dt(MS_CAP)), np.minimum(cout, dt(MS_CAP))).astype(dt)
        cnew = np.zeros((idx.size, E + 1), dtype=dt)
        valid_c = g.cn_edge < E
        cnew[:, g.cn_edge[valid_c]] = cout[:, valid_c]
        if arith == "fp64":
            # moved messages of every variable's edges [F', n, dv, 3]; the
            # posterior sums all of them, the extrinsic value of an edge all
            # but its own (exclusion sets, as in decoders.py)
            ev = g.vn_edge                                              # [n, dv]
            mv = np.where((moves[np.minimum(ev, E - 1)] & vn_valid[:, :, None])[None],
                          cnew[:, ev][..., None], 0.0)
            post = L0[None] + mv.sum(axis=2)
            other = ~np.eye(ev.shape[1], dtype=bool)                    # [t, r]: r != t
            excl = np.where(other[None, None, :, :, None], mv[:, :, None, :, :], 0.0).sum(axis=3)
            ext = np.empty((idx.size, E, 3), dtype=dt)
            ext[:, ev[vn_valid], :] = (L0[None, :, None, :] + excl)[:, vn_valid, :]
        else:
            post = _beliefs_fp32(g, L0, cnew)
            own = np.where(moves[None, :, :], cnew[:, :E, None], dt(0.0))
            ext = np.where(moves[None, :, :], post[:, g.e_var, :] - own, post[:, g.e_var, :]).astype(dt)
        vnew = np.empty((idx.size, E + 1), dtype=dt)
        vnew[:, :E] = scalarize(ext, g.e_pauli[None, :], sckind)
        vnew[:, E] = np.inf
        e_x, e_z = hard_decision(post)
        r_new = s_i ^ symplectic_syndrome(g.sx, g.sz, e_x, e_z)
        v2c[idx] = vnew
        gamma[idx] = post
        xh[idx] = e_x
        zh[idx] = e_z
        sres[idx] = r_new
        iters[idx] = ell
        done = ~r_new.any(axis=1)
        if early_exit:
            conv[idx[done]] = True
            active[idx[done]] = False
        else:
            conv[idx] = done
        if trace:
            rounds.append(dict(frames=idx.copy(), c2v=cnew[:, :E].copy(), v2c=vnew[:, :E].copy(),
                               gamma=post.copy(), gain=gain.copy(), sres=r_new.copy()))
    return JointResult(xh, zh, iters, conv, gamma, rounds if trace else None)


def judge_joint(sx, sz, ex, ez, xhat, zhat, converged) -> np.ndarray:
    """Failure: not converged, or the residual E xor E_hat is not in the
    stabilizer group (the rowspace of [S_x | S_z]); plain rank test."""
    s = np.hstack([np.asarray(sx, dtype=np.uint8), np.asarray(sz, dtype=np.uint8)])
    base = gf2.rank(s)
    rx = np.asarray(ex, dtype=np.uint8) ^ np.asarray(xhat, dtype=np.uint8)
    rz = np.asarray(ez, dtype=np.uint8) ^ np.asarray(zhat, dtype=np.uint8)
    fail = ~np.asarray(converged, dtype=bool)
    for f in range(rx.shape[0]):
        if fail[f]:
            continue
        r = np.concatenate([rx[f], rz[f]])
        if r.any() and gf2.rank(np.vstack([s, r[None, :]])) > base:
            fail[f] = True
    return fail


def logical_operators(sx, sz) -> np.ndarray:
    """A basis of the normalizer modulo the stabilizer group, as symplectic
    rows (x | z) [2k, 2n]: the vectors commuting with every row, picked
    independent of the rows and of each other."""
    sx = np.asarray(sx, dtype=np.uint8)
    sz = np.asarray(sz, dtype=np.uint8)
    n = sx.shape[1]
    # v = (vx | vz) commutes with row (sx | sz) iff sx . vz + sz . vx = 0
    comm = np.hstack([sz, sx])
    normalizer = gf2.nullspace(comm)
    acc = np.hstack([sx, sz])
    acc_rank = gf2.rank(acc)
    picked = []
    for v in normalizer:
        trial = np.vstack([acc, v[None, :]])
        r = gf2.rank(trial)
        if r > acc_rank:
            acc, acc_rank = trial, r
            picked.append(v)
    return np.array(picked, dtype=np.uint8).reshape(len(picked), 2 * n)


def judge_joint_logical(lops, ex, ez, xhat, zhat, converged) -> np.ndarray:
    """Failure: not converged, or the residual anticommutes with a logical
    operator of `lops` (rows (x | z)); equal to judge_joint when converged."""
    lops = np.asarray(lops, dtype=np.int64)
    n = lops.shape[1] // 2
    rx = np.asarray(ex, dtype=np.int64) ^ np.asarray(xhat, dtype=np.int64)
    rz = np.asarray(ez, dtype=np.int64) ^ np.asarray(zhat, dtype=np.int64)
    # <L, r> = L_x . r_z + L_z . r_x
    anti = ((rz @ lops[:, :n].T + rx @ lops[:, n:].T) & 1).any(axis=1) if lops.size else \
        np.zeros(rx.shape[0], dtype=bool)
    return ~np.asarray(converged, dtype=bool) | anti


__all__ = ["PauliGraph", "gb_joint", "depolarizing_prior", "hard_decision", "scalarize", "decode_joint",
           "judge_joint", "logical_operators", "judge_joint_logical", "symplectic_syndrome", "pauli_of",
           "BP_PHI_FLOOR", "JointResult"]
