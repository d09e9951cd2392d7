"""GPU tests of riga_eigs_batched: uneven rIGA instances solved concurrently
(one HIP stream per worker) give exactly the eigenvalues of solving each
instance alone, and match the dense oracle."""
import sys

import numpy as np
import pytest

import workloads
from oracle import assembly, eigen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _riga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_08167_amd import riga
    riga.lib()
    return riga


def _instances(count=6, seed=7):
    """Small uneven instances drawn like the 64-instance batch workload
    (ne, p, s, log-normal(0, 0.5)) but with ne in 10..30."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        out.append(workloads.small(2, int(rng.integers(10, 31)), int(rng.integers(2, 5)),
                                   int(rng.choice([4, 8])), 12, 0.5, seed=seed * 1000 + i))
    return out


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_batched_equals_individual_and_oracle(precision):
    riga = _riga()
    ws = _instances()
    probs = []
    for w in ws:
        kappa, rho = w.coefficients()
        probs.append(riga.assemble(w.dim, w.ne, w.p, w.s, kappa, rho))
    print("batch", [w.name for w in ws], flush=True)
    res = riga.eigs_batched(probs, 12, precision=precision, workers=4)
    for w, pr, (lam, U, r, st) in zip(ws, probs, res):
        lam1, U1, r1, st1 = pr.eigs(12, precision=precision)
        assert np.array_equal(lam, lam1), w.name
        kappa, rho = w.coefficients()
        Ko, Mo = assembly.assemble(w.dim, w.ne, w.p, w.s, kappa, rho)
        lr = eigen.dense_eigh(Ko, Mo)[0][:12]
        assert np.max(np.abs(lam - lr) / lr) <= 1e-10, w.name
        assert eigen.residual(Ko, Mo, lam, U.cpu().numpy()).max() <= 1e-9


def test_batched_rejects_duplicates():
    riga = _riga()
    pr = riga.assemble(2, 12, 2, 4)
    with pytest.raises(riga.RigaError) as e:
        riga.eigs_batched([pr, pr], 4)
    assert e.value.code == riga.RIGA_EINVAL
