"""The autotuner of the reduced-precision RBF block product V = K P: it
records one tile shape per column count, and every shape it may pick gives
the product within the Gram precision's elementwise bound of the float64
oracle (|V - K P|_i <= c sum_j |K_ij| |P_ij|, c = 2e-5 for float32 Gram
tiles, 5e-4 for bf16x3), the tail tiles of a ragged column count included."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from workloads import batched_cv  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2110_02820_amd as nys  # noqa: E402

DEV = "cuda"
BOUND = {nys.NYS_PREC_FP32_REFINE64: 2e-5, nys.NYS_PREC_BF16X3_REFINE64: 5e-4}


def _data(n=3000):
    w = batched_cv(n=n, with_omega=False, with_ragged=False)
    X = np.asarray(w["X"], dtype=np.float32)
    return X, w["sigma"]


def _check_product(op, X, sigma, P, prec, mu=0.0):
    V = nys.nys_op_apply(op, mu, torch.as_tensor(P, device=DEV), prec=prec).cpu().numpy().astype(np.float64)
    K = oracle.rbf_kernel_block(X.astype(np.float64), X.astype(np.float64), sigma)
    Pd = P.astype(np.float64)
    ref = K @ Pd + mu * Pd
    scale = np.abs(K) @ np.abs(Pd) + mu * np.abs(Pd)
    err = np.abs(V - ref) / scale
    assert err.max() <= BOUND[prec], (prec, P.shape[1], err.max(), np.unravel_index(err.argmax(), err.shape))


@pytest.mark.parametrize("prec", [nys.NYS_PREC_FP32_REFINE64, nys.NYS_PREC_BF16X3_REFINE64])
def test_autotune_records_shapes_that_match_the_oracle(prec, tmp_path):
    X, sigma = _data()
    n = X.shape[0]
    op = nys.Operator.rbf(torch.as_tensor(X, device=DEV), sigma)
    nys.nys_autotune_clear()
    ks = [8, 40, 130]
    nys.nys_autotune(op, prec, ks)
    assert nys.nys_autotune_entries() == len(ks)
    rng = np.random.default_rng(5)
    for k in ks + [5, 37]:
        reg, cf, bpc, fr, tuned = nys.nys_autotune_query(op, prec, k)
        assert tuned
        P = rng.standard_normal((n, k)).astype(np.float32)
        _check_product(op, X, sigma, P, prec, mu=0.3)
    path = tmp_path / "tune.txt"
    nys.nys_autotune_save(str(path))
    assert len([l for l in path.read_text().splitlines() if l.startswith("rbf_kv")]) == len(ks)
    nys.nys_autotune_clear()


@pytest.mark.parametrize("prec", [nys.NYS_PREC_FP32_REFINE64, nys.NYS_PREC_BF16X3_REFINE64])
def test_every_tile_shape_matches_the_oracle(prec, tmp_path):
    """Each shape the tuner may choose, forced through a cache file, on column
    counts that leave a ragged tail tile (k = 23 and 150)."""
    X, sigma = _data(2000)
    n = X.shape[0]
    op = nys.Operator.rbf(torch.as_tensor(X, device=DEV), sigma)
    mode = 0 if prec == nys.NYS_PREC_BF16X3_REFINE64 else 1
    rng = np.random.default_rng(6)
    for k in (23, 150):
        P = rng.standard_normal((n, k)).astype(np.float32)
        for reg, cf, fr in ((1, 1, 1), (1, 2, 1), (1, 4, 1), (0, 8, 1), (0, 16, 1), (0, 8, 2), (0, 16, 2)):
            for bpc in (4, 16):
                path = tmp_path / "force.txt"
                path.write_text("rbf_kv %d 16 %d %d %d %d %d 1.0 %d\n" % (n, mode, k, reg, cf, bpc, fr))
                nys.nys_autotune_clear()
                nys.nys_autotune_load(str(path))
                assert nys.nys_autotune_query(op, prec, k) == (bool(reg), cf, bpc, fr, True)
                _check_product(op, X, sigma, P, prec)
    nys.nys_autotune_clear()
