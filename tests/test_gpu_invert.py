"""Batched inversion through the C interface (qax_invert): the Gauss-Jordan
elimination with partial pivoting that inverts the self blocks for the
block-diagonal preconditioner (Section 6), applied to seeded random complex
Gaussian matrices.  Unlike the self blocks, which are diagonally dominant
(their LU permutation is the identity), these need row interchanges at almost
every step, so the pivot search, the interchanges of the panel and sibling
columns and the final column interchanges are all exercised.

* a heterogeneous batch of ragged orders (1 to 300) in one call, every entry
  against numpy's inverse, to 3 cond(A) eps in the norm of the inverse;
* single matrices of orders 2048, 2050, 4100 and 8192 (the largest), sampled
  columns of A X - I relative to |A| |x_j|, to 8 n eps;
* FP64 and the FP32 path of the mixed preconditioner;
* an empty batch and argument errors.
"""
import numpy as np
import pytest
import scipy.linalg as sla

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2606_31380_amd import qax  # noqa: E402

DEV = torch.device("cuda", 0)
EPS = {qax.QAX_FP64: 2.2e-16, qax.QAX_MIXED: 1.2e-7}


def rand_mats(orders, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for n in orders]


def gpu_invert(mats, prec):
    flat = np.concatenate([m.ravel() for m in mats])
    t = torch.from_numpy(flat).to(DEV)
    h = qax.qax_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        qax.qax_invert(h, prec, [m.shape[0] for m in mats], t)
    finally:
        qax.qax_destroy(h)
    out = t.cpu().numpy()
    res, o = [], 0
    for m in mats:
        n = m.shape[0]
        res.append(out[o:o + n * n].reshape(n, n))
        o += n * n
    return res


def test_random_matrices_need_pivoting():
    (a,) = rand_mats([64], 11)
    p, _, _ = sla.lu(a)
    assert int(np.sum(np.argmax(p, axis=0) != np.arange(64))) > 32


@pytest.mark.parametrize("prec", [qax.QAX_FP64, qax.QAX_MIXED])
def test_ragged_batch(prec):
    orders = [1, 3, 17, 64, 100, 127, 128, 129, 255, 300, 2, 16]
    mats = rand_mats(orders, 5)
    got = gpu_invert(mats, prec)
    for a, x in zip(mats, got):
        want = np.linalg.inv(a)
        err = np.linalg.norm(x - want) / np.linalg.norm(want)
        # forward error of an inverse: a modest multiple of cond(A) eps
        tol = 3 * np.linalg.cond(a) * EPS[prec]
        print(prec, a.shape[0], err, tol)
        assert err < tol


@pytest.mark.parametrize("prec,n", [(qax.QAX_FP64, 2048), (qax.QAX_FP64, 2050), (qax.QAX_FP64, 4100),
                                    (qax.QAX_FP64, 8192), (qax.QAX_MIXED, 2050), (qax.QAX_MIXED, 8192)])
def test_large_sampled_columns(prec, n):
    (a,) = rand_mats([n], n)
    (x,) = gpu_invert([a], prec)
    assert np.all(np.isfinite(x))
    cols = np.random.default_rng(1).choice(n, 6, replace=False)
    na = np.linalg.norm(a)
    for j in cols:
        e = np.zeros(n, dtype=complex)
        e[j] = 1.0
        r = np.linalg.norm(a @ x[:, j] - e) / (na * np.linalg.norm(x[:, j]))
        print(prec, n, j, r)
        assert r < 8 * n * EPS[prec]


def test_empty_batch_and_argument_errors():
    t = torch.zeros(16, dtype=torch.complex128, device=DEV)
    h = qax.qax_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        qax.qax_invert(h, qax.QAX_FP64, [], t)
        for orders in ([0], [8193], [4, -1]):
            with pytest.raises(qax.QaxError):
                qax.qax_invert(h, qax.QAX_FP64, orders, t)
        with pytest.raises(qax.QaxError):
            qax.qax_invert(h, 7, [4], t)
    finally:
        qax.qax_destroy(h)
