"""Serving loop on the GPU: continuous batching of many solves.

Checks that (1) every request's result in the mix is bitwise identical to the
same request solved alone, with and without the multi-request SpMM launches, (2) the admitted requests never exceed the HBM
budget at any instant and are admitted in FIFO order, (3) requests run
concurrently when budget and slots allow, (4) a request larger than the budget
is refused with ARR_ENOMEM, (5) the served results are the right eigenpairs
(dense diagonalization on small problems)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1507_06078_amd import arr, workloads as W


def make_requests():
    reqs = []
    rng = np.random.default_rng(7)
    for i in range(7):
        if i % 2 == 0:
            m = int(rng.integers(24, 40))
            A = W.laplacian_2d_potential(m, potential_seed=100 + i)
        else:
            m = int(rng.integers(9, 13))
            A = W.laplacian_3d(m, potential_seed=100 + i)
        k = int(rng.integers(5, 16))
        w = k + max(4, round(0.2 * k))
        tol = 1e-8 if i % 3 == 0 else 1e-10
        prec = arr.MIXED if i % 2 else arr.FP64
        reqs.append((A, k, w, tol, prec))
    return reqs


def handle(A, k, w, tol, prec):
    o = arr.arr_options_default()
    o.w = w
    o.precision = prec
    o.seed = 2
    return arr.arr_create(A, A.n, k, arr.SMALLEST, tol, o)


@pytest.mark.parametrize("batch_spmm", [True, False])
def test_served_results_equal_alone_and_budget_respected(batch_spmm):
    """With batch_spmm the requests' SpMMs run in multi-request launches
    (the paired and plain forms of the 3D requests; the 2D requests' grid
    form as launches of their own on the broker's stream); the results must
    still equal the solves alone bit for bit."""
    reqs = make_requests()
    alone = []
    for (A, k, w, tol, prec) in reqs:
        h = handle(A, k, w, tol, prec)
        st = arr.arr_solve(h)
        alone.append((st,) + arr.arr_get_eigpairs(h, k, A.n))
        h.close()
    hs = [handle(*r) for r in reqs]
    fps = [arr.arr_footprint(h) for h in hs]
    budget = int(2.2 * max(fps))  # forces queuing: at most two big ones at once
    srv = arr.Server(hbm_budget_bytes=budget, max_slots=3, batch_spmm=batch_spmm)
    tickets = [srv.submit(h) for h in hs]
    status = [srv.wait(t) for t in tickets]
    times = [srv.times(t) for t in tickets]
    rounds, launches = srv.batch_stats()
    if batch_spmm:  # the 3D requests' launches went through the multi-request kernel
        assert rounds > 0 and launches > 0
    else:
        assert rounds == launches == 0
    for i, (A, k, w, tol, prec) in enumerate(reqs):
        ev, X, res = arr.arr_get_eigpairs(hs[i], k, A.n)
        assert status[i] == alone[i][0] == arr.ARR_OK
        assert np.array_equal(ev, alone[i][1]), i
        assert np.array_equal(X, alone[i][2]), i
        assert np.array_equal(res, alone[i][3]), i
        lam = np.linalg.eigvalsh(A.to_scipy().toarray())[:k]
        assert np.abs(ev - lam).max() <= 1e-9 * max(1.0, np.abs(lam).max())
    # budget and slots at every admission instant; FIFO admission order
    for i, (ts, ta, td) in enumerate(times):
        assert ts <= ta <= td
        running = [j for j, (_, a, d) in enumerate(times) if a <= ta < d]
        assert sum(fps[j] for j in running) <= budget
        assert len(running) <= 3
    admits = [t[1] for t in times]
    assert admits == sorted(admits)
    # some requests overlapped in time
    overlaps = sum(1 for i in range(len(times)) for j in range(i + 1, len(times))
                   if times[i][1] < times[j][2] and times[j][1] < times[i][2])
    assert overlaps >= 1
    srv.close()
    for h in hs:
        h.close()


def test_request_over_budget_is_refused():
    A = W.laplacian_2d(30)
    h = handle(A, 10, 14, 1e-8, arr.FP64)
    srv = arr.Server(hbm_budget_bytes=arr.arr_footprint(h) // 2, max_slots=2)
    with pytest.raises(arr.ArrError) as e:
        srv.submit(h)
    assert e.value.code == arr.ARR_ENOMEM
    srv.close()
    h.close()


def test_served_without_vectors_keeps_values():
    A = W.laplacian_2d(32)
    o = arr.arr_options_default()
    o.w = 14
    o.keep_vectors = 0
    h = arr.arr_create(A, A.n, 10, arr.SMALLEST, 1e-10, o)
    srv = arr.Server(hbm_budget_bytes=arr.arr_footprint(h) + (1 << 20), max_slots=1)
    assert srv.wait(srv.submit(h)) == arr.ARR_OK
    ev, _, res = arr.arr_get_eigpairs(h, 10, A.n, vectors=False)
    exact = W.laplacian_2d_eigenvalues(32)[:10]
    assert np.abs(ev - exact).max() <= 1e-10
    with pytest.raises(arr.ArrError):
        arr.arr_get_eigpairs(h, 10, A.n, vectors=True)
    srv.close()
    h.close()


def test_served_wide_block_stays_within_its_footprint():
    """A request whose Gram products split many ways (n = 91125, block 240,
    Krylov width up to 960): every pooled buffer stays inside the footprint
    the server reserved, and the result equals the unserved solve."""
    A = W.laplacian_3d(45, potential_seed=11)
    k, w = 200, 240
    o = arr.arr_options_default()
    o.w = w
    o.precision = arr.MIXED
    h0 = arr.arr_create(A, A.n, k, arr.SMALLEST, 1e-8, o)
    st0 = arr.arr_solve(h0)
    ev0, _, res0 = arr.arr_get_eigpairs(h0, k, A.n, vectors=False)
    h0.close()
    h = arr.arr_create(A, A.n, k, arr.SMALLEST, 1e-8, o)
    srv = arr.Server(hbm_budget_bytes=arr.arr_footprint(h) + (1 << 20), max_slots=1)
    st = srv.wait(srv.submit(h))
    srv.close()
    assert st == st0 == arr.ARR_OK
    ev, _, res = arr.arr_get_eigpairs(h, k, A.n, vectors=False)
    assert np.array_equal(ev, ev0) and np.array_equal(res, res0)
    h.close()
