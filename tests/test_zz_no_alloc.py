"""The allocation-free far field (qax_farfield_noalloc) through the C
interface, against qax_farfield on the same handle: two calls in a row, the
second with fewer directions and right-hand sides (the shared workspace keeps
the first call's contents), on a handle of three independent problems; its
size limit; FP64 agreement 1e-13 of the largest entry (only the summation
order of the partial sums differs)."""
import numpy as np
import pytest

from paper_2606_31380_amd import scenarios as sc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2606_31380_amd import qax  # noqa: E402

DEV = torch.device("cuda", 0)


def directions(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 3))
    return x / np.linalg.norm(x, axis=1)[:, None]


def test_farfield_noalloc_matches_farfield():
    s = sc.tiny(n_bodies=6, n_theta=8, shapes=(0, 1, 2), k=3.0)
    s.bodies["problem"] = [0, 0, 1, 1, 1, 2]
    s.k = np.array([3.0, 6.5, 2.0])
    with qax.Problem(s) as P:
        rng = np.random.default_rng(4)
        for n_dirs, nrhs in ((900, 3), (37, 1)):
            print(f"noalloc far field: {n_dirs} directions, {nrhs} right-hand sides", flush=True)
            mu = torch.from_numpy(rng.standard_normal(P.N * nrhs) + 1j * rng.standard_normal(P.N * nrhs)).to(DEV)
            xh = directions(n_dirs, n_dirs)
            want = torch.zeros(3 * n_dirs * nrhs, dtype=torch.complex128, device=DEV)
            qax.qax_farfield(P.h, mu, xh, want, nrhs)
            got = torch.full_like(want, complex("nan"))
            d_xh = torch.from_numpy(np.ascontiguousarray(xh)).to(DEV)
            torch.cuda.synchronize()
            qax.qax_farfield_noalloc(P.h, mu, d_xh, got, nrhs)
            torch.cuda.synchronize()
            g, w = got.cpu().numpy(), want.cpu().numpy()
            assert np.all(np.isfinite(g))
            assert np.abs(g - w).max() < 1e-13 * np.abs(w).max()
        # beyond the workspace: a clear error, nothing enqueued
        big = torch.zeros(3, dtype=torch.float64, device=DEV).reshape(1, 3)
        with pytest.raises(qax.QaxError) as e:
            lib = qax.lib()
            st = lib.qax_farfield_noalloc(P.h, qax._ptr(mu), 256, qax._ptr(big), 10000, qax._ptr(got))
            qax._check(P.h, st)
        assert e.value.status == qax.QAX_ERR_ARG
