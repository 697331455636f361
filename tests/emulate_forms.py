"""NumPy model of the reduced-precision overlap arithmetic (test helper).

Each form contracts <a|b> like Fig. 2 of the paper (E <- sum_s A_a[s]^H E
A_b[s], two complex GEMMs per site and physical index) but rounds operands
and accumulators the way the GPU kernels do, so that the precision reading
of the split-BF16 form can be checked on full-size states on the CPU.

Fixed-point forms (the kernels' split-BF16 and split-int8): each GEMM
operand is rounded to a B-bit code per row (A-operand: E, T^T) or column
(B-operand: the site tensors), cut into balanced digits; a kept set of digit
pairs is multiplied exactly; with ``acc="bf16"`` the leading pair goes to
an exact accumulator and the others to an FP32 accumulator rounded to
nearest after each instruction (K = 32 values), combined in FP64.

Floating form "R2": every FP32 operand split into three bf16 pieces of their
own exponents, the six largest piece products into one FP32 accumulator per
output, E kept in FP32 with a power-of-two rescale per site.  ``trunc_bits``
models the bf16 MFMA's summation: within one instruction, products more than
``trunc_bits`` bits below the largest product of the same output are cut
(toward zero) before the sum is rounded into the accumulator.
"""
from __future__ import annotations

import numpy as np


def random_left_canonical(m, chi, rng):
    """Left-canonical MPS with bonds min(chi, 2^min(l, m-l)) (QR of complex
    Gaussian blocks), last site normalised."""
    dims = [min(chi, 2 ** min(l, m - l)) for l in range(m + 1)]
    out = []
    for l in range(m):
        z = rng.standard_normal((dims[l] * 2, dims[l + 1])) + 1j * rng.standard_normal((dims[l] * 2, dims[l + 1]))
        q, _ = np.linalg.qr(z)
        out.append(q.reshape(dims[l], 2, dims[l + 1]))
    out[-1] = out[-1] / np.linalg.norm(out[-1])
    return out


def perturbed(mps, eps, rng):
    """A nearby left-canonical state: every site plus eps * complex noise,
    re-orthogonalised by a left-to-right QR sweep, then normalised."""
    out, carry = [], None
    for l, t in enumerate(mps):
        t = t + eps * (rng.standard_normal(t.shape) + 1j * rng.standard_normal(t.shape))
        if carry is not None:
            t = np.einsum("ab,bsc->asc", carry, t)
        dl, _, dr = t.shape
        if l + 1 < len(mps):
            q, r = np.linalg.qr(t.reshape(dl * 2, dr))
            out.append(q.reshape(dl, 2, q.shape[1]))
            carry = r
        else:
            out.append(t / np.linalg.norm(t))
    return out


def _exponent(mx, margin):
    """Smallest e with mx (1 + margin) < 2^e (0 where mx == 0)."""
    mx = np.asarray(mx, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return np.where(mx > 0, np.floor(np.log2(mx * (1.0 + margin))) + 1, 0).astype(np.int64)


def _digits(X, n, bits):
    """Balanced base-2^bits digits of the integer array X, leading first."""
    r = X.astype(np.int64)
    half, mask = 1 << (bits - 1), (1 << bits) - 1
    out = []
    for _ in range(n - 1):
        d = ((r & mask) ^ half) - half
        out.append(d.astype(np.float64))
        r = (r - d) >> bits
    out.append(r.astype(np.float64))
    return out[::-1]


class FixedPoint:
    """``pairs``: digit pairs (a, b) kept in every product; ``re2_extra``:
    pairs kept in addition in the real part of T^T conj(A) only."""

    def __init__(self, n_digits, bits, pairs, acc="exact", margin=2.0 ** -24, re2_extra=(), margin_y=None):
        self.n, self.bits, self.pairs, self.acc, self.margin = n_digits, bits, list(pairs), acc, margin
        self.margin_y = margin if margin_y is None else margin_y
        self.re2_extra = list(re2_extra)
        self.B = n_digits * bits - 1            # |code| < 2^B

    def _split(self, x, e):
        lim = 2.0 ** self.B - 1
        return _digits(np.clip(np.rint(np.ldexp(x, self.B - e)), -lim, lim), self.n, self.bits)

    def _real(self, terms, shape, pairs):
        """sum over (X digits, Y digits) terms of the kept digit products"""
        w = lambda a, b: 2.0 ** (-self.bits * (a + b))
        if self.acc == "exact":
            return sum(Xd[a] @ Yd[b] * w(a, b) for Xd, Yd in terms for (a, b) in pairs)
        hi = np.zeros(shape)
        lo = np.zeros(shape, dtype=np.float32)
        rest = sorted([p for p in pairs if p != (0, 0)], key=lambda p: -(p[0] + p[1]))
        K = terms[0][0][0].shape[1]
        for k0 in range(0, K, 32):
            ks = slice(k0, k0 + 32)
            for Xd, Yd in terms:
                hi += Xd[0][:, ks] @ Yd[0][ks, :]
                for (a, b) in rest:   # one MFMA per digit pair: exact sum, one rounding
                    lo = (lo.astype(np.float64) + (Xd[a][:, ks] @ Yd[b][ks, :]) * w(a, b)).astype(np.float32)
        return hi + lo

    def cgemm(self, X, Y, conj_y):
        """X Y (or X conj(Y)) with row exponents of X and column exponents of Y."""
        ex = _exponent(np.maximum(np.abs(X.real), np.abs(X.imag)).max(1), self.margin)[:, None]
        ey = _exponent(np.maximum(np.abs(Y.real), np.abs(Y.imag)).max(0), self.margin_y)[None, :]
        Xr, Xi = self._split(X.real, ex), self._split(X.imag, ex)
        Yr, Yi = self._split(Y.real, ey), self._split(Y.imag, ey)
        neg = lambda ds: [-d for d in ds]
        if conj_y:
            re_t, im_t = [(Xr, Yr), (Xi, Yi)], [(Xi, Yr), (neg(Xr), Yi)]
        else:
            re_t, im_t = [(Xr, Yr), (Xi, neg(Yi))], [(Xr, Yi), (Xi, Yr)]
        shape = (X.shape[0], Y.shape[1])
        scale = np.ldexp(1.0, ex + ey - 2 * self.B) * 2.0 ** (2 * self.bits * (self.n - 1))
        re_pairs = self.pairs + (self.re2_extra if conj_y else [])
        return (self._real(re_t, shape, re_pairs) + 1j * self._real(im_t, shape, self.pairs)) * scale

    def overlap(self, a, b):
        E = np.ones((1, 1), dtype=np.complex128)
        for ta, tb in zip(a, b):
            En = 0
            for s in range(2):
                T = self.cgemm(E, tb[:, s, :], conj_y=False)
                En = En + self.cgemm(T.T, ta[:, s, :], conj_y=True).T
            E = En
        return complex(E[0, 0])


TEN = [(a, b) for a in range(4) for b in range(4) if a + b <= 3]
EIGHT = [(a, b) for a in range(3) for b in range(3) if a + b <= 3]
SIX = [(0, 0), (0, 1), (1, 0), (0, 2), (1, 1), (2, 0)]


def split_bf16_form():
    """The kernels' split-BF16: 31-bit codes in four balanced 8-bit digits,
    the ten pairs of weight >= 2^-24 (and (2, 2) in the real part of
    T^T conj(A)), exact leading + FP32 accumulator, FP64 combine."""
    return FixedPoint(4, 8, TEN, acc="bf16", margin=2.0 ** -30, re2_extra=[(2, 2)])


def split_i8_form():
    """The kernels' split-int8: the same digits and pairs, all sums exact."""
    return FixedPoint(4, 8, TEN, acc="exact", margin=2.0 ** -7, re2_extra=[(2, 2)])


def three_9bit_form():
    """27-bit codes in three balanced 9-bit digits (bf16 carries |n| <= 256
    exactly), the six pairs of weight >= 2^-18, exact leading accumulator."""
    return FixedPoint(3, 9, SIX, acc="bf16")


def three_9bit_eight_form():
    """27-bit codes in three balanced 9-bit digits with every product of weight
    >= 2^-27 (eight pairs) and (2, 2) in the real part of T^T conj(A): the
    cheapest fixed-point bf16 form (32 + 2 digit products per complex product
    instead of 41), with the kernels' exponent margins (2^-7 for the sliced
    rows of E and T^T, 2^-30 for the packed site columns)."""
    return FixedPoint(3, 9, EIGHT, acc="bf16", margin=2.0 ** -7, margin_y=2.0 ** -30, re2_extra=[(2, 2)])


def _bf16(x):
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32).view(np.float32).astype(np.float64)


def _mfma_sum(X, Y, trunc_bits):
    """sum_k X[:, k] Y[k, :] of bf16 values: exact, or (trunc_bits) with every
    product cut toward zero to a multiple of 2^(e - trunc_bits), 2^e <= the
    largest |product| of the same output < 2^(e+1).  Products of two bf16
    values are exact in FP32."""
    if trunc_bits is None:
        return X @ Y
    P = X.astype(np.float32)[:, :, None] * Y.astype(np.float32)[None, :, :]
    _, e = np.frexp(np.abs(P).max(axis=1, keepdims=True))
    q = np.ldexp(np.float32(1.0), e - 1 - trunc_bits).astype(np.float32)
    return (np.trunc(P / q) * q).sum(axis=1, dtype=np.float64)


class FloatingR2:
    PRODUCTS = [(0, 0), (0, 1), (1, 0), (0, 2), (2, 0), (1, 1)]

    def __init__(self, trunc_bits=None):
        self.trunc_bits = trunc_bits

    @staticmethod
    def _pieces(x):
        r, out = np.asarray(x, dtype=np.float32).astype(np.float64), []
        for _ in range(3):
            p = _bf16(r)
            out.append(p)
            r = r - p
        return out

    def _acc(self, acc, X, Y):
        Xp, Yp = self._pieces(X), self._pieces(Y)
        for k0 in range(0, X.shape[1], 32):
            ks = slice(k0, k0 + 32)
            for (a, b) in sorted(self.PRODUCTS, key=lambda p: -(p[0] + p[1])):
                acc = (acc.astype(np.float64) + _mfma_sum(Xp[a][:, ks], Yp[b][ks, :], self.trunc_bits)).astype(np.float32)
        return acc

    def overlap(self, a, b):
        Er, Ei, ex = np.ones((1, 1), np.float32), np.zeros((1, 1), np.float32), 0
        for ta, tb in zip(a, b):
            Rr = np.zeros((ta.shape[2], tb.shape[2]), np.float32)
            Ri = np.zeros_like(Rr)
            for s in range(2):
                Br, Bi = tb[:, s, :].real, tb[:, s, :].imag
                Ar, Ai = ta[:, s, :].real, ta[:, s, :].imag
                Tr = self._acc(self._acc(np.zeros((Er.shape[0], Br.shape[1]), np.float32), Er, Br), Ei, -Bi)
                Ti = self._acc(self._acc(np.zeros_like(Tr), Er, Bi), Ei, Br)
                Rr = self._acc(self._acc(Rr, Ar.T, Tr), Ai.T, Ti)     # E'_re += Ar^T Tr + Ai^T Ti
                Ri = self._acc(self._acc(Ri, Ar.T, Ti), -Ai.T, Tr)    # E'_im += Ar^T Ti - Ai^T Tr
            mx = max(np.abs(Rr).max(), np.abs(Ri).max())
            e = int(np.floor(np.log2(mx))) if mx > 0 else 0
            Er, Ei, ex = np.ldexp(Rr, -e).astype(np.float32), np.ldexp(Ri, -e).astype(np.float32), ex + e
        return complex(Er[0, 0], Ei[0, 0]) * 2.0 ** ex
