"""GPU tests of riga_factor_batched: the fronts of one tree height of many
problems in one launch per kernel give every problem exactly the
factorisation riga_factor gives it alone -- inertia, pivot counts and solves
equal bit for bit -- in FP64 and mixed precision, over problems of different
tree heights, sizes and front classes (fronts held in LDS and blocked fronts
above the LDS limit), and the solves meet the backward-error bar against the
oracle's matrices.  The batched eigensolver's first factorisations go through
the same call; its eigenvalues are checked bitwise against single solves in
test_gpu_batch.py."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from oracle import assembly, eigen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _riga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_08167_amd import riga
    riga.lib()  # raises if the library is missing: no fallback
    return riga


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# 2D and 3D, rIGA and IGA, p = 2..5: tree heights from 5 to 12 and largest
# fronts from below to well above the LDS limit (128 in FP64, 176 in FP32)
CASES = [workloads.small(2, 24, 3, 8, 10, 0.5, seed=11), workloads.small(3, 6, 2, 3, 10, 0.4, seed=12),
         workloads.small(2, 40, 3, 0, 10, 0.3, seed=13), workloads.small(3, 12, 2, 4, 10, 0.4, seed=14),
         workloads.small(2, 17, 5, 4, 10, 0.5, seed=15), workloads.small(2, 64, 2, 16, 10, 0.5, seed=16),
         workloads.small(3, 10, 3, 0, 10, 0.3, seed=17)]


def _problems(riga, cases):
    out = []
    for w in cases:
        kappa, rho = w.coefficients()
        out.append(riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho))
    return out


def _shifts(probs):
    # one shift per problem, spread over the low spectrum (between the
    # estimates of eigenvalues, so no pivot is perturbed)
    return [0.0 if i % 3 == 0 else 37.5 * (i + 1) * pr.dim for i, pr in enumerate(probs)]


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_factor_batched_equals_individual(precision):
    riga = _riga()
    probs = _problems(riga, CASES)
    info = [pr.info for pr in probs]
    assert max(i["max_front"] for i in info) > 176 and min(i["max_front"] for i in info) <= 128
    assert len({i["tree_height"] for i in info}) >= 3
    sigmas = _shifts(probs)
    rng = np.random.default_rng(5)
    bs = [torch.tensor(rng.standard_normal(pr.n_dof), dtype=torch.float64, device="cuda") for pr in probs]
    _say("batched factorisation", [w.name for w in CASES], sigmas, "precision", precision)
    batched = riga.factor_batched(probs, sigmas, precision=precision)
    xb = [pr.solve(b).cpu().numpy() for pr, b in zip(probs, bs)]
    for w, pr, sg, b, x, (neg, st) in zip(CASES, probs, sigmas, bs, xb, batched):
        _say("single", w.name, sg)
        neg1, st1 = pr.factor(sg, precision=precision)
        x1 = pr.solve(b).cpu().numpy()
        assert neg == neg1, w.name
        assert st["n_2x2_pivots"] == st1["n_2x2_pivots"] and st["n_perturbed_pivots"] == 0, w.name
        assert np.array_equal(x, x1), (w.name, np.max(np.abs(x - x1)))
        if precision == 0:
            kappa, rho = w.coefficients()
            Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
            assert neg == eigen.inertia(Ko, Mo, sg), w.name
            A = (Ko - sg * Mo).tocsr()
            bh = b.cpu().numpy()
            r = bh - A @ x
            berr = np.linalg.norm(r) / (sp.linalg.norm(A, 1) * np.linalg.norm(x) + np.linalg.norm(bh))
            assert berr <= 1e-12, (w.name, berr)


def test_factor_batched_with_complex_hermitian_pencils():
    """Real and complex Hermitian pencils (the magnetic Laplacian in its
    real-equivalent form, 2 x 2 blocks) in one batched call: each equals its
    single factorisation bit for bit (inertia and solve)."""
    riga = _riga()
    probs = [riga.assemble(2, 16, 2, 4, potential=(1.0, 0.5)), _problems(riga, CASES[:1])[0],
             riga.assemble(3, 6, 2, 3, potential=(0.3, -0.7, 1.1))]
    assert probs[0].hermitian and probs[2].hermitian
    sigmas = [40.0, 0.0, 60.0]
    out = riga.factor_batched(probs, sigmas)
    rng = np.random.default_rng(8)
    bs = [torch.tensor(rng.standard_normal(pr.n_dof), dtype=torch.float64, device="cuda") for pr in probs]
    xb = [pr.solve(b).cpu().numpy() for pr, b in zip(probs, bs)]
    for pr, sg, b, x, (neg, st) in zip(probs, sigmas, bs, xb, out):
        neg1, _ = pr.factor(sg)
        assert neg == neg1
        assert np.array_equal(x, pr.solve(b).cpu().numpy())


def test_factor_batched_repeated_and_reordered():
    """Two batched calls in a row over the same problems in another order
    and at other shifts: each factorisation depends only on its problem and
    shift."""
    riga = _riga()
    probs = _problems(riga, CASES[:5])
    sig1 = [10.0 * (i + 1) for i in range(5)]
    riga.factor_batched(probs, sig1)
    order = [3, 0, 4, 1, 2]
    sig2 = [sig1[i] * 2.0 for i in order]
    out = riga.factor_batched([probs[i] for i in order], sig2)
    b = {i: torch.ones(probs[i].n_dof, dtype=torch.float64, device="cuda") for i in range(5)}
    xb = {i: probs[i].solve(b[i]).cpu().numpy() for i in order}
    for q, i in enumerate(order):
        neg1, _ = probs[i].factor(sig2[q])
        assert out[q][0] == neg1
        assert np.array_equal(xb[i], probs[i].solve(b[i]).cpu().numpy())


def test_factor_batched_singular_instance():
    """One instance factorised exactly on an eigenvalue: RIGA_ESINGULAR for
    the call, its perturbed pivot counted, the others unaffected."""
    riga = _riga()
    from test_gpu_parity import _unit_pencil_n1
    pr0, sigma = _unit_pencil_n1(riga)
    others = _problems(riga, CASES[:2])
    with pytest.raises(riga.RigaError) as e:
        riga.factor_batched([others[0], pr0, others[1]], [0.0, sigma, 0.0])
    assert e.value.code == riga.RIGA_ESINGULAR
    out = riga.factor_batched([others[0], pr0, others[1]], [0.0, sigma, 0.0], allow_singular=True)
    assert [o[1]["n_perturbed_pivots"] for o in out] == [0, 1, 0]
    assert out[1][0] == 0 and out[1][1]["status"] == riga.RIGA_ESINGULAR
    assert out[0][0] == 0 and out[2][0] == 0


def test_factor_batched_rejects_bad_arguments():
    riga = _riga()
    probs = _problems(riga, CASES[:2])
    assert riga.factor_batched([], []) == []
    for bad in ([probs[0], probs[0]], [0.0, 0.0]), (probs, [0.0, float("nan")]):
        with pytest.raises(riga.RigaError) as e:
            riga.factor_batched(*bad)
        assert e.value.code == riga.RIGA_EINVAL
    with pytest.raises(riga.RigaError) as e:
        riga.factor_batched(probs, [0.0, 0.0], precision=7)
    assert e.value.code == riga.RIGA_EINVAL
