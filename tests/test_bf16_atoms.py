"""The BF16 form ranks atoms by BF16 correlations.  Its BF16 atom is the FP32
product of the FP32-rounded 1D table entries, rounded to BF16 (the constant
atoms 1/N).  Kernels that build atoms from the tables on the fly rely on the
constant atom coming out as exactly 1/N from the product as well; this pins
that for every block size and both families, from the oracle's FP64 tables."""
import numpy as np
import pytest

from oracle import aqmp_oracle as O


def _bf16_rne(x32: np.ndarray) -> np.ndarray:
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


@pytest.mark.parametrize("n", [4, 8, 16, 32, 64])
@pytest.mark.parametrize("table", ["dct", "haar"])
def test_constant_atom_product_is_one_over_n_in_bf16(n, table):
    t = (O.dct_matrix(n) if table == "dct" else O.haar_matrix(n)).astype(np.float32)
    prod = (t[0][:, None] * t[0][None, :]).astype(np.float32)   # fl32(T32[0][y] * T32[0][x])
    want = _bf16_rne(np.array([1.0 / n], dtype=np.float32))[0]
    assert np.all(_bf16_rne(prod) == want)


def test_bf16_rounding_helper_is_round_to_nearest_even():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa (1.0) wins;
    # 1 + 3 * 2^-8 rounds up to 1 + 2^-6
    x = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9], dtype=np.float32)
    got = _bf16_rne(x)
    assert got.tolist() == [0x3F80, 0x3F82, 0x3F80]
