"""The split-bf16 product of the bf16 models' backward, emulated on the CPU.

An fp32 value x is taken as hi = bf16(x) (round to nearest even) and
lo = bf16(x - hi); a product a b as hi(a) hi(b) + hi(a) lo(b) + lo(a) hi(b).
Fixed by the arithmetic: x - hi is exact in fp32 with at most 16 significant
bits and |x - hi| <= 2^-8 |x|, so lo keeps its top 8 and |x - hi - lo| <= 2^-17
|x|; the dropped lo(a) lo(b) is at most 2^-16 |a b| and the two residuals
2^-17 |a b| each, so one product is within 2^-15 of a b, while plain bf16
operands leave up to 2^-7.  These are the bounds the backward's products rely
on (checked on the GPU against fp32 products and the FP64 oracle)."""
import numpy as np


def bf16(x):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def split(x):
    x = np.asarray(x, dtype=np.float32)
    hi = bf16(x)
    lo = bf16(x - hi)
    return hi, lo


def test_bf16_rounding_examples():
    # exactly representable values stay; halfway cases go to the even neighbour
    assert bf16(np.float32(1.0)) == 1.0
    assert bf16(np.float32(1.0 + 2.0 ** -8)) == 1.0                  # tie -> even (1.0)
    assert bf16(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6  # tie -> even
    assert bf16(np.float32(1.0 + 2.0 ** -7)) == 1.0 + 2.0 ** -7


def test_split_represents_fp32_to_2e_minus_17():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(200_000) * np.exp(rng.uniform(-20, 20, 200_000))).astype(np.float32)
    hi, lo = split(x)
    err = np.abs(x.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64))
    assert np.all(err <= 2.0 ** -17 * np.abs(x.astype(np.float64)))
    assert np.all(np.abs(lo) <= 2.0 ** -8 * np.abs(hi))             # at most half of hi's last bit


def test_three_products_within_2e_minus_16_and_plain_bf16_not():
    rng = np.random.default_rng(1)
    a = rng.standard_normal(100_000).astype(np.float32)
    b = rng.standard_normal(100_000).astype(np.float32)
    ah, al = split(a)
    bh, bl = split(b)
    d = lambda v: v.astype(np.float64)
    exact = d(a) * d(b)
    three = d(ah) * d(bh) + d(ah) * d(bl) + d(al) * d(bh)
    plain = d(ah) * d(bh)
    rel3 = np.abs(three - exact) / np.abs(exact)
    rel1 = np.abs(plain - exact) / np.abs(exact)
    assert rel3.max() <= 2.0 ** -15 * 1.01
    assert rel1.max() > 2.0 ** -10           # plain bf16 is two orders of magnitude off
    # a dot product of 512 terms (exact accumulation): relative to sum |a b|
    k = 512
    A = rng.standard_normal((64, k)).astype(np.float32)
    B = rng.standard_normal((k, 64)).astype(np.float32)
    Ah, Al = split(A)
    Bh, Bl = split(B)
    ref = d(A) @ d(B)
    got = d(Ah) @ d(Bh) + d(Ah) @ d(Bl) + d(Al) @ d(Bh)
    scale = np.abs(d(A)) @ np.abs(d(B))
    assert np.max(np.abs(got - ref) / scale) <= 2.0 ** -15 * 1.01
