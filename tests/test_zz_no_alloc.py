"""The no-allocation inversion entry point (cq_slater_inverse_static) against the allocating
one (cq_slater_inverse): the same inverse, log|det| and sign on two calls in a row, the second
smaller, and a batch beyond the static workspace rejected with CQ_EINVAL."""
import numpy as np
import pytest

import paper_2209_14487_amd as cq

pytestmark = pytest.mark.gpu


def well_conditioned(rng, nmat, n):
    A = rng.uniform(-1, 1, (nmat, n, n))
    return A + n ** 0.5 * np.eye(n)[None] * rng.choice([-1.0, 1.0], (nmat, 1, 1))


def both(A, dtype):
    nmat, n = A.shape[0], A.shape[1]
    out = []
    for f in (cq.slater_inverse, cq.slater_inverse_static):
        tA = cq.DeviceArray(A.astype(dtype))
        tM = cq.DeviceArray(shape=A.shape, dtype=dtype)
        tl = cq.DeviceArray(shape=(nmat,), dtype=np.float64)
        ts = cq.DeviceArray(shape=(nmat,), dtype=np.int32)
        f(tA, tM, tl, ts)
        out.append((tM.numpy(), tl.numpy(), ts.numpy()))
    return out


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_static_workspace_inverse_equals_the_allocating_one(dtype):
    rng = np.random.default_rng(17)
    # blocked path (n > 64, ragged last block), then a smaller batch on the LDS path (n <= 64)
    for n, nmat in ((200, 9), (40, 5)):
        A = well_conditioned(rng, nmat, n)
        (M0, l0, s0), (M1, l1, s1) = both(A, dtype)
        assert np.array_equal(M0, M1) and np.array_equal(l0, l1) and np.array_equal(s0, s1), (n, nmat)
        ref_s, ref_l = np.linalg.slogdet(A.astype(dtype).astype(np.float64))
        assert np.array_equal(s1, ref_s.astype(np.int32))
        assert np.all(np.abs(l1 - ref_l) <= 1e-11 * np.maximum(1.0, np.abs(ref_l)))


def test_static_workspace_reports_a_singular_matrix_then_recovers():
    rng = np.random.default_rng(18)
    A = well_conditioned(rng, 4, 80)
    A[1, 5] = A[1, 9]
    tA = cq.DeviceArray(A)
    tM = cq.DeviceArray(shape=A.shape, dtype=np.float64)
    tl = cq.DeviceArray(shape=(4,), dtype=np.float64)
    ts = cq.DeviceArray(shape=(4,), dtype=np.int32)
    with pytest.raises(cq.CqError) as ei:
        cq.slater_inverse_static(tA, tM, tl, ts)
    assert ei.value.status == cq.CQ_ESINGULAR and "matrix 0 or 1" in str(ei.value)
    # the status words left in the shared workspace are cleared by the next call
    B = well_conditioned(rng, 3, 80)
    (M0, l0, _), (M1, l1, _) = both(B, "float64")
    assert np.array_equal(M0, M1) and np.array_equal(l0, l1)


def test_static_workspace_rejects_a_batch_beyond_its_size():
    n = 1024
    nmat = 64  # 64 x 8 MiB > 64 MiB
    A = cq.DeviceArray(shape=(1, 16), dtype=np.float64)  # never read: the size check comes first
    with pytest.raises(cq.CqError) as ei:
        cq.lib()
        st = cq.lib().cq_slater_inverse_static(A.ptr, 8, n, nmat, A.ptr, A.ptr, A.ptr, None)
        cq._check(st)
    assert ei.value.status == cq.CQ_EINVAL and "static workspace" in str(ei.value)
