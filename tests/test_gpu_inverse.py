"""GPU parity of the batched FP64 Slater inverse (cq_slater_inverse: the periodic-recompute
kernels applied to caller-held matrices) against LAPACK through numpy: inverse, log|det| and
sign, for the one-workgroup LDS path (n <= 64) and the blocked path (n > 64, with a ragged last
block and a panel narrower than 4 columns at n = 101; one and two panel rows per thread of the
register panel at n = 600 and 1040, 8-column panels above n = 1024), FP64 and FP32 storage, an odd
number of matrices, and a singular matrix reported."""
import numpy as np
import pytest

import paper_2209_14487_amd as cq

pytestmark = pytest.mark.gpu


def well_conditioned(rng, nmat, n):
    A = rng.uniform(-1, 1, (nmat, n, n))
    return A + n ** 0.5 * np.eye(n)[None] * rng.choice([-1.0, 1.0], (nmat, 1, 1))


@pytest.mark.parametrize("n,nmat", [(4, 3), (32, 17), (100, 5), (101, 3), (256, 4), (600, 3), (1040, 2)])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_slater_inverse_matches_lapack(n, nmat, dtype):
    rng = np.random.default_rng(n * 7 + nmat)
    A = well_conditioned(rng, nmat, n)
    A = A.astype(dtype).astype(np.float64)  # the stored values are the reference's input
    tA = cq.DeviceArray(A.astype(dtype))
    tM = cq.DeviceArray(shape=A.shape, dtype=dtype)
    tl = cq.DeviceArray(shape=(nmat,), dtype=np.float64)
    ts = cq.DeviceArray(shape=(nmat,), dtype=np.int32)
    cq.slater_inverse(tA, tM, tl, ts)
    M = tM.numpy().astype(np.float64)
    ld, sg = tl.numpy(), ts.numpy()
    ref_s, ref_l = np.linalg.slogdet(A)
    inv = np.linalg.inv(A)
    tol = 1e-11 if dtype == "float64" else 2e-7
    for m in range(nmat):
        # Minv[m][a][j] = (A^-1)[j][a]
        err = np.abs(M[m] - inv[m].T).max() / np.abs(inv[m]).max()
        assert err < tol, (m, err)
    assert np.all(np.abs(ld - ref_l) <= 1e-11 * np.maximum(1.0, np.abs(ref_l)))
    assert np.array_equal(sg, ref_s.astype(np.int32))


def test_slater_inverse_reports_a_singular_matrix():
    rng = np.random.default_rng(5)
    n, nmat = 80, 6
    A = well_conditioned(rng, nmat, n)
    A[3, 7] = A[3, 2]  # two equal rows in matrix 3
    tA = cq.DeviceArray(A)
    tM = cq.DeviceArray(shape=A.shape, dtype=np.float64)
    tl = cq.DeviceArray(shape=(nmat,), dtype=np.float64)
    ts = cq.DeviceArray(shape=(nmat,), dtype=np.int32)
    with pytest.raises(cq.CqError) as ei:
        cq.slater_inverse(tA, tM, tl, ts)
    assert ei.value.status == cq.CQ_ESINGULAR
    assert "matrix 2 or 3" in str(ei.value)


def paired_blocks(n, delta, dtype):
    """2 x 2 blocks on rows and columns (t, t + h), h = n // 2: [[delta, 1], [1, 1]] for even t,
    [[1, 1], [1, delta]] for odd t (a last odd row is 1 on the diagonal).  Column t of A^T then
    holds delta in row t and 1 in row t + h for even t, so only the largest-magnitude pivot is
    usable; rows t and t + h lie in different waves of the panel kernel and of the small kernel."""
    h = n // 2
    A = np.zeros((n, n))
    for t in range(h):
        a, b = (delta, 1.0) if t % 2 == 0 else (1.0, delta)
        A[t, t], A[t, t + h], A[t + h, t], A[t + h, t + h] = a, 1.0, 1.0, b
    if n % 2:
        A[n - 1, n - 1] = 1.0
    return A.astype(dtype).astype(np.float64)


@pytest.mark.parametrize("n", [40, 300, 602, 1024, 1041])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_slater_inverse_takes_the_largest_pivot_across_waves(n, dtype):
    """A pivot of 1e-20 sits below the n eps max|A| threshold: picking it instead of the 1 in the
    other row of its block would report the matrix singular (and lose the inverse)."""
    A = np.stack([paired_blocks(n, 1e-20, dtype), paired_blocks(n, 1e-20, dtype).T])
    nmat = A.shape[0]
    tA = cq.DeviceArray(A.astype(dtype))
    tM = cq.DeviceArray(shape=A.shape, dtype=dtype)
    tl = cq.DeviceArray(shape=(nmat,), dtype=np.float64)
    ts = cq.DeviceArray(shape=(nmat,), dtype=np.int32)
    cq.slater_inverse(tA, tM, tl, ts)
    M = tM.numpy().astype(np.float64)
    ref_s, ref_l = np.linalg.slogdet(A)
    inv = np.linalg.inv(A)
    tol = 1e-14 if dtype == "float64" else 1e-7
    for m in range(nmat):
        assert np.abs(M[m] - inv[m].T).max() <= tol * np.abs(inv[m]).max(), m
    assert np.all(np.abs(tl.numpy() - ref_l) <= 1e-12)
    assert np.array_equal(ts.numpy(), ref_s.astype(np.int32))
