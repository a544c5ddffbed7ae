"""H and S from caller-given coefficients (hsbuild_forward_coefficients): the
FP64 path against the oracle's Eqs. 4-5 on arbitrary coefficients, and the
split path's exactness: coefficients that fit in five 8-bit slices per column
scale, with lambda = 1 and T = 1 (so the right operands are the left one),
must give the FP64 product to FP64 rounding."""
import numpy as np
import pytest
import torch

from flapw_cells import make_case
from oracle import hs_oracle as o

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    yield


def _full(M):
    return np.triu(M) + np.triu(M, 1).conj().T


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_fp64_from_random_coefficients():
    from paper_1712_07206_amd.hsbuild import HSBuilder
    case = make_case(1, n_g=700)
    rng = np.random.default_rng(5)
    shape = (case["n_atoms"], 2, case["n_l"], 700)
    coef = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    b = HSBuilder.from_case(case)
    H, S = b.forward_from_coefficients(torch.as_tensor(coef, device="cuda"), torch.as_tensor(case["T"], device="cuda"))
    Hr, Sr = o.hamiltonian(case, coef), o.overlap(case, coef)
    assert rel(_full(H.cpu().numpy()), Hr) <= 1e-13
    assert rel(_full(S.cpu().numpy()), Sr) <= 1e-13


@pytest.mark.parametrize("prec_name", ["bf16", "fp16"])
def test_split_exact_for_forty_bit_inputs(prec_name):
    from paper_1712_07206_amd import HSB_SPLIT_BF16, HSB_SPLIT_FP16
    from paper_1712_07206_amd.hsbuild import HSBuilder
    prec = HSB_SPLIT_BF16 if prec_name == "bf16" else HSB_SPLIT_FP16
    case = dict(make_case(1, n_g=640))
    n, n_at, n_l = 640, case["n_atoms"], case["n_l"]
    case["udot_norm2"] = np.ones_like(case["udot_norm2"])  # lambda = 1
    m = 2 * n_l
    case["T"] = np.stack([np.eye(m, dtype=np.complex128)] * case["n_types"])  # Y = W
    rng = np.random.default_rng(8)
    e = rng.integers(-3, 4, n)  # per-column binary exponent
    mant = rng.integers(-(2 ** 40) + 1, 2 ** 40, size=(n_at, 2, n_l, n, 2)).astype(np.float64)
    coef = (mant[..., 0] + 1j * mant[..., 1]) * np.ldexp(1.0, e - 40)[None, None, None, :]
    b = HSBuilder.from_case(case, precision=prec, n_slices=5)
    H, S = b.forward_from_coefficients(torch.as_tensor(coef, device="cuda"), torch.as_tensor(case["T"], device="cuda"))
    Sr = o.overlap(case, coef)
    Hs, Ss = _full(H.cpu().numpy()), _full(S.cpu().numpy())
    eh, es = rel(Hs, Sr), rel(Ss, Sr)
    print("split %s on 40-bit inputs: rel err H %.3e S %.3e" % (prec_name, eh, es))
    assert eh <= 1e-14 and es <= 1e-14
