"""The allocation-free Gram entry point (arr_gram_noalloc) against arr_gram,
through the C ABI, on two calls in a row, the second with a smaller input
(the shared scratch array keeps the first call's partials, so this also checks
that nothing stale is read). Both are checked against an FP64 product on the
CPU within the forward error bound of a length-n dot product,
gamma_n sum_l |x_li y_lj|."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1507_06078_amd import arr

U = 2.0 ** -53


def _case(n, mx, my, dtype, same, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = torch.randn((n, mx), generator=g, dtype=torch.float64)
    Y = X if same else torch.randn((n, my), generator=g, dtype=torch.float64)
    Xd = X.to(dtype).cuda()
    Yd = Xd if same else Y.to(dtype).cuda()
    return Xd, Yd


def _check(Xd, Yd, fp32_cores=False):
    mx, my = Xd.shape[1], Yd.shape[1]
    G1 = torch.full((mx, my), np.nan, dtype=torch.float64, device="cuda")
    G2 = torch.full((mx, my), np.nan, dtype=torch.float64, device="cuda")
    arr.arr_gram(Xd, Yd, G1, fp32_cores=fp32_cores)
    arr.arr_gram_noalloc(Xd, Yd, G2, fp32_cores=fp32_cores)
    torch.cuda.synchronize()
    x, y = Xd.double().cpu().numpy(), Yd.double().cpu().numpy()
    ref = x.T @ y
    n = x.shape[0]
    # FP32 cores: products of FP32 data summed in FP32 within 32-row slices
    u = 2.0 ** -24 if fp32_cores else U
    bound = 1.01 * (n * u / (1 - n * u)) * (np.abs(x).T @ np.abs(y)) + 1e-300
    g1, g2 = G1.cpu().numpy(), G2.cpu().numpy()
    assert np.isfinite(g2).all()
    assert np.all(np.abs(g2 - ref) <= bound)
    assert np.all(np.abs(g2 - g1) <= 2 * bound)
    if Xd.data_ptr() == Yd.data_ptr():
        np.testing.assert_array_equal(g2, g2.T)  # symmetric product: upper triangle mirrored exactly
    return g1, g2


def test_noalloc_gram_matches_gram_two_calls_second_smaller():
    # first call: the benchmark's 240-column symmetric Gram on 200000 rows (many split partials)
    Xd, _ = _case(200_000, 240, 240, torch.float64, True, 1)
    _check(Xd, Xd)
    # second call, smaller: FP32 data, rectangular, ragged widths
    Xs, Ys = _case(5_003, 30, 47, torch.float32, False, 2)
    _check(Xs, Ys)
    # and a third on FP32 matrix cores
    _check(Xs, Ys, fp32_cores=True)


def test_noalloc_gram_rejects_products_beyond_the_scratch():
    """mx * my above 2^22 doubles: ARR_EINVAL before any launch."""
    Xd = torch.zeros((64, 2049), dtype=torch.float64, device="cuda")
    Yd = torch.zeros((64, 2049), dtype=torch.float64, device="cuda")
    G = torch.zeros((2049, 2049), dtype=torch.float64, device="cuda")
    with pytest.raises(arr.ArrError) as e:
        arr.arr_gram_noalloc(Xd, Yd, G)
    assert e.value.code == arr.ARR_EINVAL and "scratch" in str(e.value)
