"""The dense layers' matrix-core products (gm_mlp_gemm: the forward X W^T,
the backward dZ W and the weight gradient dZ^T X) element by element against
FP64 products of the same BF16 operands.

Bar: |C - C_64| <= 1e-5 sum_k |A_ik B_kj| per element.  The device sums BF16
products exactly inside each 32-deep matrix-core step and adds the steps (and
the K splits of the weight gradient) in FP32, so its error is a few FP32
roundings of the running sums, bounded by about (K / 32) 2^-24 sum |A B|
(6e-6 at K = 4096); an operand read from the wrong row, column or tile edge
moves an element by a large fraction of that sum.

Shapes: the network's (in 1056, hidden 512, out 16, batches of 4096 rows and
ragged row counts), with row gathers, sizes that are not multiples of the
64 x 64 output tile or the 32-deep K slice, and K = 0.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import mlp as M
from paper_2404_07780_amd import gmfit as G

RTOL = 1e-5


def _op(rng, shape, scale=1.0):
    return M.bf16(rng.normal(scale=scale, size=shape))


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda().to(torch.bfloat16)


def _check(got, a, b, tag):
    ref = a @ b
    bound = RTOL * (np.abs(a) @ np.abs(b)) + 1e-30
    ratio = np.abs(got.astype(np.float64) - ref) / bound
    print(f"{tag}: worst {ratio.max():.3f} of the bar, median {np.median(ratio):.3g}", flush=True)
    assert np.all(ratio <= 1.0), (tag, np.unravel_index(np.argmax(ratio), ratio.shape), ratio.max())


@pytest.mark.parametrize("m,n,k", [(4096, 512, 1056), (300, 512, 1056), (4096, 16, 512), (77, 24, 40), (8, 8, 8)])
def test_forward_product(m, n, k):
    rng = np.random.default_rng(m + n + k)
    a, b = _op(rng, (m, k)), _op(rng, (n, k), 0.05)
    got = G.gm_mlp_gemm(G.GEMM_NT, _dev(a), _dev(b)).cpu().numpy()
    _check(got, a, b.T, f"NT {m}x{n}x{k}")


def test_forward_product_gathered_rows():
    rng = np.random.default_rng(5)
    a, b = _op(rng, (5000, 1056)), _op(rng, (512, 1056), 0.05)
    rows = rng.permutation(5000)[:1000].astype(np.int32)
    got = G.gm_mlp_gemm(G.GEMM_NT, _dev(a), _dev(b), a_rows=torch.from_numpy(rows).cuda()).cpu().numpy()
    _check(got, a[rows], b.T, "NT gathered")


@pytest.mark.parametrize("m,n,k", [(4096, 512, 512), (300, 512, 16), (4096, 1056, 512), (70, 40, 24)])
def test_backward_product(m, n, k):
    rng = np.random.default_rng(m * 3 + n + k)
    a, b = _op(rng, (m, k), 1e-3), _op(rng, (k, n), 0.05)
    got = G.gm_mlp_gemm(G.GEMM_NN, _dev(a), _dev(b)).cpu().numpy()
    _check(got, a, b, f"NN {m}x{n}x{k}")


@pytest.mark.parametrize("m,n,k", [(512, 1056, 4096), (512, 512, 4096), (16, 512, 4096), (512, 1056, 1000),
                                   (64, 64, 300), (24, 40, 70), (8, 8, 0)])
def test_weight_gradient_product(m, n, k):
    rng = np.random.default_rng(m + 7 * n + k)
    if k == 0:
        e = torch.empty(0, m, dtype=torch.bfloat16, device="cuda")
        assert torch.all(G.gm_mlp_gemm(G.GEMM_TN, e, e) == 0.0)
        return
    a, b = _op(rng, (k, m), 1e-3), _op(rng, (k, n))
    got = G.gm_mlp_gemm(G.GEMM_TN, _dev(a), _dev(b)).cpu().numpy()
    _check(got, a.T, b, f"TN {m}x{n}x{k}")


def test_weight_gradient_gathered_rows_and_determinism():
    rng = np.random.default_rng(9)
    a, b = _op(rng, (4096, 512), 1e-3), _op(rng, (8192, 1056))
    rows = rng.permutation(8192)[:4096].astype(np.int32)
    rd = torch.from_numpy(rows).cuda()
    ad, bd = _dev(a), _dev(b)
    got = G.gm_mlp_gemm(G.GEMM_TN, ad, bd, b_rows=rd)
    _check(got.cpu().numpy(), a.T, b[rows], "TN gathered")
    # the K splits are added in a fixed order: the same call gives the same bits,
    # and the gather equals the product of the gathered copy
    assert torch.equal(got, G.gm_mlp_gemm(G.GEMM_TN, ad, bd, b_rows=rd))
    assert torch.equal(got, G.gm_mlp_gemm(G.GEMM_TN, ad, _dev(b[rows])))


def test_invalid_shapes_are_rejected():
    x = _dev(np.zeros((16, 12)))
    y = _dev(np.zeros((16, 16)))
    with pytest.raises(G.GmError) as e:
        G.gm_mlp_gemm(G.GEMM_NT, x, x)            # k = 12 is not a multiple of 8
    assert e.value.code == G.GM_EINVAL
    with pytest.raises(G.GmError) as e:
        G.gm_mlp_gemm(G.GEMM_TN, x, y)            # m = 12 is not a multiple of 8
    assert e.value.code == G.GM_EINVAL
    with pytest.raises(G.GmError) as e:
        G.gm_mlp_gemm(G.GEMM_TN, y, y, a_rows=torch.zeros(16, dtype=torch.int32, device="cuda"))
    assert e.value.code == G.GM_EINVAL
