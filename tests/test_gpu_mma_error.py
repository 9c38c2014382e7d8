"""The matrix cores' accumulation against exact sums (the assumption behind the fast-score
error bound).  One 32 x 32 block of e4m3 code products over K = 256 (the c5 dimension)
runs on the BF16 matrix cores (codes widened to BF16, exact) and on the FP8 matrix cores
(codes as they are), FP32 accumulation in both.  Code products are multiples of 2^-18
below 2^18, so the K-term sums are exact in FP64 in any order.

The BF16 path must stay inside the library's model, |c - S| <= 2 gamma_{K+2}(2^-24)
sum |terms| (the factor 2 covers the unspecified internal order); the FP8 path is
measured and reported (it is why FP8 data is multiplied on the BF16 matrix cores)."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

K = 256


def _gamma(n, u=2.0 ** -24):
    return n * u / (1 - n * u)


def _codes(g, shape, kind):
    """e4m3 codes (no NaN codes 0x7f / 0xff) of a given value pattern."""
    if kind == "uniform":        # every finite code, both signs
        c = g.integers(0, 254, size=shape)
        return np.where(c >= 0x7f, c + 1, c).astype(np.uint8)
    if kind == "spread":         # large magnitudes mixed with subnormals
        big = g.integers(0x68, 0x7f, size=shape)          # 2^6 .. 448
        small = g.integers(0x01, 0x08, size=shape)        # subnormals m 2^-9
        c = np.where(g.random(shape) < 0.5, big, small)
        return (c | (g.integers(0, 2, size=shape) << 7)).astype(np.uint8)
    if kind == "cancel":         # pairs of equal large terms of opposite sign, then small ones
        c = g.integers(0x60, 0x7f, size=shape).astype(np.uint8)
        half = shape[1] // 2
        c[:, half:half + half // 2] = c[:, :half // 2] | 0x80
        c[:, half + half // 2:] = g.integers(0x01, 0x20, size=(shape[0], shape[1] - half - half // 2))
        return c
    raise ValueError(kind)


def _ratios(R, kind, a, b):
    av, bv = O._fp8_codes_f64(a), O._fp8_codes_f64(b)
    exact = av @ bv.T
    absum = np.abs(av) @ np.abs(bv).T
    got = R.rkmips_diag_mma_probe(kind, a, b).astype(np.float64)
    assert np.all(np.isfinite(got))
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(absum > 0, np.abs(got - exact) / absum, 0.0)
    return float(r.max())


@pytest.mark.parametrize("pattern", ["uniform", "spread", "cancel"])
def test_bf16_matrix_cores_accumulate_like_fp32_and_fp8_measured(pattern):
    from paper_2211_12751_amd import rkmips as R
    g = np.random.default_rng({"uniform": 1, "spread": 2, "cancel": 3}[pattern])
    bound = 2.0 * _gamma(K + 2)
    worst_bf16, worst_fp8, worst_f8k64 = 0.0, 0.0, 0.0
    print(f"\n[case] mma probe pattern={pattern} K={K}", flush=True)
    for trial in range(8):
        a, b = _codes(g, (32, K), pattern), _codes(g, (32, K), pattern)
        worst_bf16 = max(worst_bf16, _ratios(R, 0, a, b))
        worst_fp8 = max(worst_fp8, _ratios(R, 1, a, b))
        worst_f8k64 = max(worst_f8k64, _ratios(R, 2, a, b))
    lg = lambda x: f"2^{np.log2(x):.1f}" if x > 0 else "0"
    print(f"[mma] {pattern}: max |c - S| / sum|terms|  BF16 path {worst_bf16:.3e} ({lg(worst_bf16)})  "
          f"FP8 path {worst_fp8:.3e} ({lg(worst_fp8)})  FP8 K=64 path {worst_f8k64:.3e} ({lg(worst_f8k64)})  "
          f"model bound {bound:.3e} ({lg(bound)})", flush=True)
    assert worst_bf16 <= bound
    # the 32x32x64 instruction with the operand layout the seed pass uses: a wrong layout
    # or scale would leave sums far from the exact ones
    assert worst_f8k64 <= 2.0 ** -8


def test_hardware_fp8_conversion_decodes_ocp_e4m3():
    """The canonical FP8 rescoring decodes item codes with the hardware conversion: every
    code (each in all four byte positions of a word) must give the format's value, and the
    two NaN codes NaN."""
    from paper_2211_12751_amd import rkmips as R
    print("\n[case] fp8 hardware decode, 256 codes x 4 byte positions", flush=True)
    codes = np.arange(256, dtype=np.uint8)
    words = np.stack([np.roll(codes, s) for s in range(4)], axis=1).ravel()   # every code at every position
    got = R.rkmips_diag_fp8_decode(words).astype(np.float64)
    want = O._fp8_codes_f64(words)
    nan = (words & 0x7f) == 0x7f
    assert np.all(np.isnan(got[nan]))
    assert np.array_equal(got[~nan], want[~nan])
    # signed zeros keep their sign
    assert np.signbit(got[words == 0x80]).all() and not np.signbit(got[words == 0x00]).any()
