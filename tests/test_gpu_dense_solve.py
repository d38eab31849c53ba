"""GPU tests of the setup's batched dense solve (amamg_dense_solve: the local block systems of
the wirebasket interpolation and the exact coarsest-level inverse) against numpy.linalg.solve.

Cases cover every launch path: one workgroup per system (n <= 64, or n <= 256 with 32 or more
systems), and the panel / interchange / tile launches with the panel rows in registers (1 to 4
row groups at width 16, 8 row groups at width 8) and in global memory past 2048 rows; ragged last
panels; matrices built so that a
row interchanged out of a panel is chosen again as a pivot in the same panel (the interchanges
are applied to the other columns afterwards, in order); singular systems, which report their
first zero pivot column without disturbing the other systems.  Bar: relative solution error
<= 1e-11 per system (partial pivoting on Gaussian matrices; numpy's LAPACK pivots by another
modulus, so the factors differ by rounding only)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def systems(rng, nsys, n, nrhs):
    A = rng.standard_normal((nsys, n, n)) + 1j * rng.standard_normal((nsys, n, n))
    B = rng.standard_normal((nsys, n, nrhs)) + 1j * rng.standard_normal((nsys, n, nrhs))
    return A, B


def check(lib, ctx, A, B, bound=1e-11):
    aug = np.concatenate([A, B], axis=2)
    out, info = ctx.dense_solve(aug)
    n = A.shape[1]
    for s in range(A.shape[0]):
        x = out[s, :, n:]
        ref = np.linalg.solve(A[s], B[s])
        err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
        assert info[s] == 0 and err <= bound, (s, info[s], err)
    return out, info


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n,nrhs,nsys", [
    (8, 8, 64),        # one workgroup per system (small n)
    (168, 32, 40),     # one workgroup per system (n <= 256, >= 32 systems), ragged last panel
    (200, 5, 3),       # panel launches, rows in one register group
    (600, 40, 2),      # three, two and one register groups
    (300, 7, 33),      # n > 256 with many systems: panel launches
    (1100, 3, 1),      # panels of width 8 in registers while more than 1024 rows remain
    (2100, 2, 1),      # panels in global memory past 2048 rows, then width 8, then width 16
])
def test_batched_dense_solve_matches_numpy(lib, ctx, n, nrhs, nsys):
    say("dense solve", n, nrhs, nsys)
    A, B = systems(np.random.default_rng(n + nsys), nsys, n, nrhs)
    check(lib, ctx, A, B)


def repeated_pivot_matrix(rng, n, k0):
    """A matrix whose factorisation chooses row p as the pivot of column k0, sends row k0 to
    position p, and then chooses position p again for column k0 + 1 (and likewise a second
    pair two columns later): the same row leaves the panel twice."""
    A = 0.01 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    for k, p in ((k0, n - 3), (k0 + 2, n - 7)):
        A[p, k], A[p, k + 1] = 10.0, 1.0           # pivot of column k
        A[k, k], A[k, k + 1] = 1.0, 100.0          # after the swap and elimination: 99.9 at p
    for i in range(n):
        A[i, i] += 0.05                             # keep later pivots away from zero
    return A


@pytest.mark.parametrize("n,nsys,k0", [(40, 1, 0), (40, 32, 5), (130, 2, 18), (300, 1, 33)])
def test_a_row_chosen_twice_within_a_panel(lib, ctx, n, nsys, k0):
    say("repeated pivots", n, nsys, k0)
    rng = np.random.default_rng(7 + n)
    A = np.stack([repeated_pivot_matrix(rng, n, k0) for _ in range(nsys)])
    B = rng.standard_normal((nsys, n, 6)) + 1j * rng.standard_normal((nsys, n, 6))
    check(lib, ctx, A, B)


@pytest.mark.parametrize("n,nsys", [(40, 3), (200, 3), (120, 40)])
def test_singular_system_reports_its_zero_pivot_column(lib, ctx, n, nsys):
    say("singular", n, nsys)
    rng = np.random.default_rng(99)
    A, B = systems(rng, nsys, n, 4)
    A[1, :, 21] = 0.0                               # column 21 of system 1 vanishes
    out, info = ctx.dense_solve(np.concatenate([A, B], axis=2))
    assert info[1] == 22
    for s in range(nsys):
        if s == 1:
            continue
        ref = np.linalg.solve(A[s], B[s])
        assert info[s] == 0
        assert np.linalg.norm(out[s, :, n:] - ref) / np.linalg.norm(ref) <= 1e-11


def test_dense_solve_arguments_are_checked(lib, ctx):
    with pytest.raises(lib.AmamgError) as e:
        ctx.dense_solve(np.zeros((1, 0, 1), dtype=complex))
    assert e.value.status == lib.STATUS_CODES["INVALID_ARG"]
