"""Autotuner and every launch choice it can make, through the C interface.

Each pair-sum workgroup size / source-chunk schedule / right-hand sides per
pass and each block-apply load width is set by hand (qax_set_tuning) and the
result checked against the oracle (FP64 1e-12, FP32 1e-5 relative) and
against the default choice; qax_autotune must pick supported choices, keep
results unchanged and reproduce them from its cache file.
"""
import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import pairsum as opair
from paper_2606_31380_amd import scenarios as sc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2606_31380_amd import qax  # noqa: E402

DEV = torch.device("cuda", 0)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def scenario():
    # uneven bodies of three shapes, two independent problems
    s = sc.random_mixed(n_bodies=12, side=12.0, k=3.0, seed=5)
    b = s.bodies.copy()
    b["problem"][6:] = 1
    return sc.Scenario("tune", b, np.array([3.0, 5.5]), s.dirs)


@pytest.fixture(scope="module")
def ref():
    s = scenario()
    d = geo.discretize(s)
    n = d.pos.shape[0]
    rng = np.random.default_rng(1)
    mu = rng.standard_normal((n, 5)) + 1j * rng.standard_normal((n, 5))
    tg = np.sort(rng.choice(n, 300, replace=False))
    want = np.stack([opair.pair_sum(d, s.k, mu[:, r], targets=tg) for r in range(5)], 1)
    return s, mu, tg, want


def run_pair(P, prec, mu):
    nrhs = mu.shape[1]
    out = P.vec(nrhs)
    qax.qax_pair_sum(P.h, prec, torch.from_numpy(np.ascontiguousarray(mu.ravel())).to(DEV), out, nrhs)
    return out.cpu().numpy().reshape(-1, nrhs)


@pytest.mark.parametrize("tpb", [128, 256, 512])
@pytest.mark.parametrize("mult", [1, 4, 16])
def test_pair_sum_every_schedule(ref, tpb, mult):
    s, mu, tg, want = ref
    with qax.Problem(s) as P:
        qax.qax_set_tuning(P.h, pair_tpb=(tpb, tpb), pair_slot_mult=(mult, mult),
                           pair_nrc=((2, 2, 2, 2), (2, 2, 2, 2)))
        assert qax.qax_tuning(P.h)["pair_tpb"]["fp32"] == tpb
        got = run_pair(P, qax.QAX_FP64, mu[:, :1])
        assert rel(got[tg, 0], want[:, 0]) < 1e-12
        got = run_pair(P, qax.QAX_MIXED, mu[:, :1])
        assert rel(got[tg, 0], want[:, 0]) < 1e-5
        assert np.abs(got[tg, 0] - want[:, 0]).max() < 1e-5 * np.abs(want[:, 0]).max()
        got = run_pair(P, qax.QAX_FP64, mu)
        assert rel(got[tg], want) < 1e-12


def test_reciprocal_every_super_task_size(ref):
    # one right-hand side: the reciprocal kernels with 1, 2, 4 and 8 block
    # pairs per super-task side (different launch counts and slot layouts),
    # each against the oracle, element by element
    s, mu, tg, want = ref
    with qax.Problem(s) as P:
        for sv in (1, 2, 4, 8):
            qax.qax_set_tuning(P.h, pair_sym_s=(sv, sv))
            assert qax.qax_tuning(P.h)["pair_sym_s"] == {"fp64": sv, "fp32": sv}
            got = run_pair(P, qax.QAX_FP64, mu[:, :1])[tg, 0]
            assert np.abs(got - want[:, 0]).max() < 1e-12 * np.abs(want[:, 0]).max()
            got = run_pair(P, qax.QAX_MIXED, mu[:, :1])[tg, 0]
            assert rel(got, want[:, 0]) < 1e-5
            assert np.abs(got - want[:, 0]).max() < 1e-5 * np.abs(want[:, 0]).max()
            assert np.abs(got - want[:, 0]).max() < 1e-5 * np.abs(want[:, 0]).max()
        with pytest.raises(qax.QaxError):
            qax.qax_set_tuning(P.h, pair_sym_s=(9, 1))


@pytest.mark.parametrize("nrc", [1, 2, 4, 8, 16, 32])
def test_pair_sum_every_rhs_pass(ref, nrc):
    s, mu, tg, want = ref
    with qax.Problem(s) as P:
        n64 = min(nrc, 8)
        tpb32 = 128 if nrc == 32 else 256      # 32 per pass fits LDS with 128 targets
        qax.qax_set_tuning(P.h, pair_tpb=(256, tpb32), pair_nrc=((n64,) * 4, (nrc,) * 4))
        assert rel(run_pair(P, qax.QAX_FP64, mu)[tg], want) < 1e-12
        assert rel(run_pair(P, qax.QAX_MIXED, mu)[tg], want) < 1e-5
        assert np.abs(run_pair(P, qax.QAX_MIXED, mu)[tg] - want).max() < 1e-5 * np.abs(want).max()


def test_unsupported_choices_rejected():
    with qax.Problem(scenario()) as P:
        for kw in ({"pair_tpb": (96, 256)}, {"pair_slot_mult": (0, 8)},
                   {"pair_nrc": ((16, 8, 8, 8), (4, 8, 16, 16))},
                   {"pair_tpb": (256, 512), "pair_nrc": ((4, 8, 8, 8), (4, 8, 16, 16))},
                   {"gemv_vec": (4, 1)}):
            with pytest.raises(qax.QaxError):
                qax.qax_set_tuning(P.h, **kw)
        # the handle still works with its previous choices
        assert qax.qax_tuning(P.h)["pair_tpb"]["fp64"] == 256


def test_block_apply_every_width():
    s = scenario()
    rng = np.random.default_rng(2)
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        v = torch.from_numpy(rng.standard_normal(P.N) + 1j * rng.standard_normal(P.N)).to(DEV)
        outs = {}
        for vec64, vec32 in ((1, 1), (2, 2), (2, 4)):
            qax.qax_set_tuning(P.h, gemv_vec=(vec64, vec32))
            for inv, prec in ((0, qax.QAX_FP64), (1, qax.QAX_FP64), (1, qax.QAX_MIXED)):
                o = P.vec()
                qax.qax_block_apply(P.h, inv, prec, v, o, 1)
                outs.setdefault((inv, prec), []).append(o.cpu().numpy())
        for (inv, prec), lst in outs.items():
            tol = 1e-14 if prec == qax.QAX_FP64 else 1e-6
            for o in lst[1:]:
                assert rel(o, lst[0]) < tol


def test_autotune_and_cache(ref, tmp_path):
    s, mu, tg, want = ref
    cache = tmp_path / "tune.txt"
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        qax.qax_autotune(P.h, nrhs_max=5, cache_path=str(cache))
        t = qax.qax_tuning(P.h)
        assert t["tuned"] and not t["from_cache"]
        assert t["pair_tpb"]["fp64"] in (128, 256, 512) and t["pair_tpb"]["fp32"] in (128, 256, 512)
        assert t["pair_ms"]["fp32"] > 0 and t["default_pair_ms"]["fp32"] > 0
        assert rel(run_pair(P, qax.QAX_FP64, mu)[tg], want) < 1e-12
        assert rel(run_pair(P, qax.QAX_MIXED, mu)[tg], want) < 1e-5
        assert np.abs(run_pair(P, qax.QAX_MIXED, mu)[tg] - want).max() < 1e-5 * np.abs(want).max()
    assert cache.read_text().startswith("qax-tune v2 ")
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)     # same signature: built and assembled
        qax.qax_autotune(P.h, nrhs_max=5, cache_path=str(cache))
        t2 = qax.qax_tuning(P.h)
        assert t2["from_cache"]
        for key in ("pair_tpb", "pair_slot_mult", "pair_nrc", "gemv_vec", "pair_sym_s"):
            assert t2[key] == t[key]
        assert rel(run_pair(P, qax.QAX_MIXED, mu)[tg], want) < 1e-5
        assert np.abs(run_pair(P, qax.QAX_MIXED, mu)[tg] - want).max() < 1e-5 * np.abs(want).max()


def test_autotune_single_rhs_not_slower_than_default(ref):
    s, mu, tg, want = ref
    with qax.Problem(s) as P:
        qax.qax_autotune(P.h, nrhs_max=1)
        t = qax.qax_tuning(P.h)
        for prec in ("fp64", "fp32"):       # the default is one of the candidates
            assert t["pair_ms"][prec] <= 1.15 * t["default_pair_ms"][prec]
            assert t["pair_sym_s"][prec] in (1, 2, 4, 8)
        assert rel(run_pair(P, qax.QAX_MIXED, mu[:, :1])[tg, 0], want[:, 0]) < 1e-5
        assert np.abs(run_pair(P, qax.QAX_MIXED, mu[:, :1])[tg, 0] - want[:, 0]).max() < 1e-5 * np.abs(want[:, 0]).max()


def test_solve_after_tuning_matches_default():
    s = sc.tiny(n_bodies=3, n_panels=1, n_theta=8, k=2.0, spacing=2.5)
    dirs = np.array([[0.0, 0.0, 1.0]])
    xs = []
    for tune in (False, True):
        with qax.Problem(s) as P:
            qax.qax_assemble_self(P.h)
            if tune:
                qax.qax_autotune(P.h, nrhs_max=1)
            x = P.vec()
            qax.qax_solve(P.h, qax.QAX_FP64, dirs, x, 1, tol=1e-12, maxit=200)
            xs.append(x.cpu().numpy())
    assert rel(xs[1], xs[0]) < 1e-11
    assert math.isfinite(float(np.abs(xs[1]).sum()))
