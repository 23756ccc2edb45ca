"""The arithmetic behind the matrix-core pieces forms, emulated on the CPU
(numpy's float16 and a bf16 rounding written here), independent of the HIP
code: a float32 value split into rounded pieces, and the float32 product
re-formed from the piece products that the kernels issue.

* two fp16 pieces (hi, lo), each the round-to-nearest fp16 of what is left:
  for a set whose largest magnitude m lies in [2^-2, 2^14) every value is
  kept to within 2^-22 of itself plus the lo piece's subnormal step 2^-25
  (2^-23 of m); the products hi hi + hi lo + lo hi reproduce a b to within
  about 2^-21 relative plus that floor;
* three bf16 pieces (hi, mid, lo): every normal float32 value kept to within
  2^-24 relative; the six products of weight >= 2^-24 reproduce a b to
  within a few float32 roundings.
"""
import numpy as np

F16_FLOOR = 2.0 ** -25


def f16_split2(x):
    """hi + lo, each the round-to-nearest fp16 of what the earlier piece left
    (numpy rounds float32 -> float16 to nearest, ties to even)."""
    x = np.asarray(x, np.float32)
    hi = x.astype(np.float16)
    lo = (x - hi.astype(np.float32)).astype(np.float16)
    return hi.astype(np.float64), lo.astype(np.float64)


def bf16_rn(x):
    """Round float32 to bf16 (nearest, ties to even), as float32."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def bf16_split3(x):
    x = np.asarray(x, np.float32)
    h = bf16_rn(x)
    r1 = (x - h).astype(np.float32)
    m = bf16_rn(r1)
    lo = bf16_rn((r1 - m).astype(np.float32))
    return h.astype(np.float64), m.astype(np.float64), lo.astype(np.float64)


def _sets(rng, n_sets=400, n=160):
    """Value sets like a model's folded coefficients or a row's features:
    a largest magnitude m in [2^-2, 2^14), the rest spread over six decades
    below it, both signs."""
    m = 2.0 ** rng.uniform(-2, 14, n_sets)
    mag = m[:, None] * 10.0 ** rng.uniform(-6, 0, (n_sets, n))
    mag[:, 0] = m * (1 - 2 ** -12)
    return (mag * rng.choice([-1.0, 1.0], (n_sets, n))).astype(np.float32), m


def test_f16_two_pieces_keep_22_bits():
    rng = np.random.default_rng(7)
    x, m = _sets(rng)
    hi, lo = f16_split2(x)
    xd = x.astype(np.float64)
    err = np.abs(xd - (hi + lo))
    assert np.all(np.abs(hi) <= 65504.0)
    assert np.all(err <= 2.0 ** -22 * np.abs(xd) + F16_FLOOR)
    # the floor is 2^-23 of the set's largest value at worst
    assert np.all(F16_FLOOR <= 2.0 ** -23 * m)


def test_f16_three_piece_products_reproduce_float32_products():
    rng = np.random.default_rng(11)
    a, ma = _sets(rng)
    b, mb = _sets(rng)
    ha, la = f16_split2(a)
    hb, lb = f16_split2(b)
    ab = a.astype(np.float64) * b.astype(np.float64)
    got = ha * hb + ha * lb + la * hb
    bound = 2.0 ** -21 * np.abs(ab) + F16_FLOOR * (np.abs(a) + np.abs(b)) + F16_FLOOR ** 2
    assert np.all(np.abs(got - ab) <= bound)
    # a dot product over a row of features and a model's coefficients: the
    # error stays within 2^-21 of the sum of the products' magnitudes
    dot, ref = got.sum(1), ab.sum(1)
    scale = np.abs(ab).sum(1) + F16_FLOOR * (np.abs(a) + np.abs(b)).sum(1)
    assert np.all(np.abs(dot - ref) <= 2.0 ** -21 * scale)


def test_f16_split_outside_the_range_needs_the_scale():
    # the fold scales a set whose largest value reaches 2^14 (fp16 overflows
    # past 65504) and the kernel undoes the power of two exactly
    x = np.float32(3.0e5)
    with np.errstate(over="ignore"):
        hi, _ = f16_split2(x)
    assert np.isinf(hi)
    e = int(np.frexp(np.float64(x))[1]) - 14     # brings x to [2^13, 2^14)
    hi, lo = f16_split2(np.ldexp(x, -e).astype(np.float32))
    assert 2.0 ** 13 <= abs(hi) < 2.0 ** 14
    back = np.ldexp(hi + lo, e)
    assert abs(back - float(x)) <= 2.0 ** -22 * float(x)


def test_bf16_three_pieces_and_six_products():
    rng = np.random.default_rng(13)
    a, _ = _sets(rng)
    b, _ = _sets(rng)
    pa, pb = bf16_split3(a), bf16_split3(b)
    ad = a.astype(np.float64)
    assert np.all(np.abs(ad - sum(pa)) <= 2.0 ** -24 * np.abs(ad))
    ab = ad * b.astype(np.float64)
    pairs = ((0, 0), (0, 1), (1, 0), (0, 2), (1, 1), (2, 0))
    got = sum(pa[i] * pb[j] for i, j in pairs)
    assert np.all(np.abs(got - ab) <= 2.0 ** -22 * np.abs(ab))
