"""Host checks of the three-piece bfloat16 split used by the sinc-DVR product
on the bf16 matrix cores (procmv_set_dvr_kernel kind 3).

Each binary32 value v is written as hi + mid + lo, with hi = v rounded to the
nearest bfloat16 (ties to even), mid = the remainder rounded likewise, lo =
what is left.  The kernel relies on three facts, checked here exhaustively
over whole binades (every binary32 significand) at several exponents and
both signs:
  * the split is exact: hi + mid + lo == v, and lo is itself a bfloat16;
  * every piece product is exact in binary32 (8-bit by 8-bit significands);
  * the three dropped products (mid lo', lo mid', lo lo') are at most
    2^-24 + 2^-24 + 2^-32 of |v v'| (|mid| <= 2^-8 |v|, |lo| <= 2^-16 |v|),
    about 2^-27 in root mean square: the rounding level of a binary32
    product.
"""
import numpy as np


def round_bf16(a):
    """Nearest bfloat16 (ties to even) of binary32 values, as binary32."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def split3(v):
    v = np.asarray(v, np.float32)
    hi = round_bf16(v)
    r1 = (v - hi).astype(np.float32)
    mid = round_bf16(r1)
    lo = (r1 - mid).astype(np.float32)
    return hi, mid, lo


def is_bf16(a):
    return np.all((np.asarray(a, np.float32).view(np.uint32) & 0xFFFF) == 0)


def binade(exponent, sign=1.0):
    """All binary32 values in [2^e, 2^(e+1))."""
    m = np.arange(1 << 23, dtype=np.uint32)
    bits = ((np.uint32(exponent + 127) << np.uint32(23)) | m).astype(np.uint32)
    return (sign * bits.view(np.float32)).astype(np.float32)


def test_split_is_exact_and_pieces_are_bfloat16():
    for e in (-100, -20, -1, 0, 5, 19, 60):
        for sign in (1.0, -1.0):
            v = binade(e, sign)
            hi, mid, lo = split3(v)
            assert is_bf16(hi) and is_bf16(mid) and is_bf16(lo)
            total = hi.astype(np.float64) + mid.astype(np.float64) + lo.astype(np.float64)
            assert np.array_equal(total, v.astype(np.float64)), (e, sign)
            # magnitudes of the pieces relative to v
            assert np.all(np.abs(mid) <= 2.0 ** -8 * np.abs(v))
            assert np.all(np.abs(lo) <= 2.0 ** -16 * np.abs(v))


def test_piece_products_exact_and_dropped_terms_small():
    rng = np.random.default_rng(5)
    # symbol-like and vector-like values over a wide range of magnitudes
    t = (rng.standard_normal(1 << 20) * np.exp(rng.uniform(-8, 14, 1 << 20))).astype(np.float32)
    x = (rng.standard_normal(1 << 20) * np.exp(rng.uniform(-30, 0, 1 << 20))).astype(np.float32)
    th, tm, tl = split3(t)
    xh, xm, xl = split3(x)
    for a in (th, tm, tl):
        for b in (xh, xm, xl):
            p32 = (a * b).astype(np.float32)
            assert np.array_equal(p32.astype(np.float64), a.astype(np.float64) * b), \
                "a product of two bfloat16 values must be exact in binary32"
    exact = t.astype(np.float64) * x.astype(np.float64)
    kept = sum(a.astype(np.float64) * b for a, b in
               ((th, xh), (th, xm), (tm, xh), (th, xl), (tl, xh), (tm, xm)))
    dropped = exact - kept
    nz = exact != 0
    ratio = np.abs(dropped[nz]) / np.abs(exact[nz])
    assert np.all(ratio <= 2.0 ** -23 + 2.0 ** -32)
    assert np.sqrt(np.mean(ratio ** 2)) < 2.0 ** -26
    # the dropped terms have either sign (rounded pieces): no one-signed bias
    frac_pos = np.mean(dropped[nz] * exact[nz] > 0)
    assert 0.4 < frac_pos < 0.6
