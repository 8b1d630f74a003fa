"""Depolarizing channel, syndromes and bit packing (test oracle).

Channel (Section II, system model): every qubit independently suffers I with
probability 1 - p and each of X, Y, Z with probability p/3.  The X part of
the error is e_x = [X or Y], the Z part e_z = [Z or Y].  For a CSS code the
trace-inner-product syndrome of the X part reduces to s = H_Z e_x over GF(2)
(Section II, syndrome definition and eq. (resid)).

Sampling layout (this project's reading; the paper fixes no generator):
  key      = (seed mod 2^32, seed >> 32)
  counter  = (q // 4, frame mod 2^32, frame >> 32, stream)
  qubit q  takes 32-bit output word (q mod 4) of that Philox4x32-10 call
  thresholds, computed in IEEE double and floored:
      T_X = floor(p/3 * 2^32), T_Y = floor((2p)/3 * 2^32), T_Z = floor(p * 2^32)
  u < T_X -> X,  T_X <= u < T_Y -> Y,  T_Y <= u < T_Z -> Z,  else I,
  so e_x = [u < T_Y] and e_z = [T_X <= u < T_Z].

Bit packing: bit b of 64-bit word w holds index 64 w + b; unused high bits
of the last word are zero.
"""
from __future__ import annotations

import math

import numpy as np

from .philox import philox4x32


def thresholds(p: float) -> tuple[int, int, int]:
    """(T_X, T_Y, T_Z) for 0 <= p < 1, each a 32-bit unsigned integer."""
    if not (0.0 <= p < 1.0):
        raise ValueError("p must lie in [0, 1)")
    two32 = 4294967296.0
    tx = math.floor((p / 3.0) * two32)
    ty = math.floor(((2.0 * p) / 3.0) * two32)
    tz = math.floor(p * two32)
    return int(tx), int(ty), int(tz)


def uniforms(seed: int, stream: int, frame0: int, nframes: int, n: int) -> np.ndarray:
    """The 32-bit draw of every (frame, qubit): uint64 array [nframes, n]."""
    frames = np.arange(frame0, frame0 + nframes, dtype=np.uint64)
    calls = (n + 3) // 4
    t = np.arange(calls, dtype=np.uint64)
    c0 = np.broadcast_to(t[None, :], (nframes, calls))
    c1 = np.broadcast_to((frames & np.uint64(0xFFFFFFFF))[:, None], (nframes, calls))
    c2 = np.broadcast_to((frames >> np.uint64(32))[:, None], (nframes, calls))
    c3 = np.uint64(stream & 0xFFFFFFFF)
    k0 = np.uint64(seed & 0xFFFFFFFF)
    k1 = np.uint64((seed >> 32) & 0xFFFFFFFF)
    out = philox4x32(c0, c1, c2, c3, k0, k1)
    u = np.stack(out, axis=-1).reshape(nframes, calls * 4)
    return u[:, :n]


def sample_paulis(seed: int, stream: int, frame0: int, nframes: int, n: int, p: float):
    """(e_x, e_z) bit planes, uint8 arrays [nframes, n]."""
    tx, ty, tz = thresholds(p)
    u = uniforms(seed, stream, frame0, nframes, n)
    ex = (u < ty).astype(np.uint8)
    ez = ((u >= tx) & (u < tz)).astype(np.uint8)
    return ex, ez


def syndrome(h, e) -> np.ndarray:
    """s = H e over GF(2), batched: e [F, n] -> s [F, m] (uint8)."""
    h = np.asarray(h, dtype=np.int64)
    e = np.asarray(e, dtype=np.int64)
    return ((e @ h.T) & 1).astype(np.uint8)


def words(nbits: int) -> int:
    return (nbits + 63) // 64


def pack(bits) -> np.ndarray:
    """[F, nbits] 0/1 -> [F, words(nbits)] uint64, bit b of word w = index 64w+b."""
    bits = np.asarray(bits, dtype=np.uint64)
    f, nb = bits.shape
    nw = words(nb)
    padded = np.zeros((f, nw * 64), dtype=np.uint64)
    padded[:, :nb] = bits & np.uint64(1)
    shifts = np.arange(64, dtype=np.uint64)
    return (padded.reshape(f, nw, 64) << shifts).sum(axis=2, dtype=np.uint64)


def unpack(packed, nbits: int) -> np.ndarray:
    """Inverse of pack: [F, words] uint64 -> [F, nbits] uint8."""
    packed = np.asarray(packed).astype(np.uint64)
    f, nw = packed.shape
    shifts = np.arange(64, dtype=np.uint64)
    bits = (packed[:, :, None] >> shifts) & np.uint64(1)
    return bits.reshape(f, nw * 64)[:, :nbits].astype(np.uint8)


def prior_llr(p: float) -> float:
    """Binary prior LLR of the X part: ln((1 - 2p/3) / (2p/3)).

    The paper's prior (Section II notation, L_0 = ln((1-e0)/(e0/3))) is the
    GF(4) scalar; the binary decoder of the X part uses the marginal
    P(e_x = 1) = P(X) + P(Y) = 2p/3.
    """
    q = 2.0 * p / 3.0
    return math.log((1.0 - q) / q)
