"""GPU block-banded preconditioner (through the C ABI) against the oracle's P."""
import numpy as np
import pytest

from paper_1709_08803_amd import workloads as W
from oracle import linear as Lin

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bim():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_1709_08803_amd import bim as B
    B.lib()
    return B


CASES = [
    ("tiny-31x11-default", lambda: W.tiny(0.7), -1),
    ("tiny-31x11-h1", lambda: W.tiny(0.7), 1),
    ("31x11-h2", lambda: W.tiny(1.4), 2),
    ("61x21-h1", lambda: W.working(0.7, N=61, M=21), 1),
    ("61x21-default", lambda: W.working(0.7, N=61, M=21), -1),
    ("ragged-45x9-h3", lambda: W.make_problem(45, 9, -12, 12, 0, 6, 0.9, [W.Bump(0.25, 1.3, 0.9)]), 3),
    ("full-31x13", lambda: W.make_problem(31, 13, -10, 10, -6, 6, 1.2, [], half_domain=False), 1),
    # surface tension: P is the preconditioner of the problem without it
    ("tension-31x11-h2", lambda: W.make_problem(31, 11, -16, 16, 0, 10, 1.4, [W.Bump(0.1, 1.0, 1.0)], tau=0.1), 2),
    ("tension-full-31x13", lambda: W.make_problem(31, 13, -10, 10, -6, 6, 1.2, [], half_domain=False, tau=0.05), 1),
    # pivot blocks of s = N + 1 = 192, the largest the register inversion holds
    ("max-block-191x5-h1", lambda: W.make_problem(191, 5, -20, 20, 0, 1, 0.9, [W.Bump(0.25, 1.3, 0.9)]), 1),
    # s = 193, 212, 300: blocks beyond the register kernel, inverted as 2 x 2 block matrices
    # (the leading 192 block and the Schur complement in registers, the rest on the matrix cores)
    ("split-block-192x5-h1", lambda: W.make_problem(192, 5, -20, 20, 0, 1, 0.9, [W.Bump(0.25, 1.3, 0.9)]), 1),
    ("split-block-211x5-h1", lambda: W.make_problem(211, 5, -40, 30, 0, 1, 0.7, [W.Bump(0.2, 1.0, 1.0)]), 1),
    ("split-block-299x5-h2", lambda: W.make_problem(299, 5, -30, 30, 0, 2, 1.2, [W.Bump(0.2, 1.0, 1.0)]), 2),
    # s = 385: the augmented-matrix Gauss-Jordan kernel beyond that
    ("big-block-384x5-h1", lambda: W.make_problem(384, 5, -40, 40, 0, 1, 0.9, [W.Bump(0.25, 1.3, 0.9)]), 1),
]


@pytest.mark.parametrize("name,mk,hb", CASES, ids=[c[0] for c in CASES])
def test_precond_apply_matches_oracle_solve(bim, name, mk, hb):
    p = mk()
    dp = bim.DeviceProblem(p)
    P = bim.Preconditioner(dp, hb)
    if hb < 0:  # the library's default band: max(1, min(10, round(M / 6))) slices
        assert P.band == max(1, min(10, round(p.M / 6)))
    pc_ref = Lin.Preconditioner(p, hb=P.band)
    rng = np.random.default_rng(5)
    for trial in range(2):
        r = rng.standard_normal(p.n_unknowns)
        z_ref = pc_ref.apply(r)
        z = P.apply(torch.as_tensor(r, device="cuda"))
        torch.cuda.synchronize()
        err = np.abs(z.cpu().numpy() - z_ref).max() / np.abs(z_ref).max()
        print(name, "precond rel err", err)
        # the diagonal blocks' conditioning grows with N (their trapezoidal x-integration
        # recurrences): 1e-9 for the 385-wide blocks, 1e-10 up to 300
        assert err <= (1e-10 if p.N + 1 <= 300 else 1e-9)
    P.close()


def test_precond_full_size_solves_banded_system(bim):
    # 181 x 61: check P z = r with the oracle's banded product (P is never formed on the CPU)
    p = W.working(0.7)
    dp = bim.DeviceProblem(p)
    P = bim.Preconditioner(dp)
    assert P.band == 10
    r = np.random.default_rng(6).standard_normal(p.n_unknowns)
    z = P.apply(torch.as_tensor(r, device="cuda"))
    torch.cuda.synchronize()
    z = z.cpu().numpy()
    res = Lin.banded_matvec(p, z, P.band) - r
    print("181x61 |Pz - r| / |r|", np.abs(res).max() / np.abs(r).max(), "bytes", P.nbytes)
    assert np.abs(res).max() <= 1e-9 * np.abs(r).max()
    P.close()


def test_precond_rejects_bad_band(bim):
    p = W.tiny(0.7)
    dp = bim.DeviceProblem(p)
    with pytest.raises(bim.BimError):
        bim.Preconditioner(dp, p.M)


def test_fp32_storage_operator_solves_the_banded_system(bim):
    """FP32 storage (half the bytes): the block elimination and block LU of P in
    FP64, then, for pivot blocks of 128 < s <= 192, both substitutions that form
    the dense Schur inverse S^-1 in FP32 on FP32 copies of the FP64 factors, and
    the other arrays the apply reads rounded to FP32.  So it is not the FP64
    operator rounded: part of the factorisation runs in FP32.  At 181 x 61 its
    apply still solves the banded system P z = r of the oracle's banded product,
    next to the FP64 one, to FP32 rounding amplified by the conditioning of the
    Schur complement (the FP32 substitutions add ~1e-6, far below that)."""
    p = W.working(0.7)
    dp = bim.DeviceProblem(p)
    r = np.random.default_rng(6).standard_normal(p.n_unknowns)
    rd = torch.as_tensor(r, device="cuda")
    P64 = bim.Preconditioner(dp)
    z64 = P64.apply(rd).cpu().numpy()
    b64 = P64.nbytes
    P64.close()
    P32 = bim.Preconditioner(dp, storage="fp32")
    assert P32.storage == "fp32" and P32.band == 10
    z32 = P32.apply(rd).cpu().numpy()
    z32b = P32.apply(rd).cpu().numpy()
    print("bytes", b64, P32.nbytes)
    assert np.array_equal(z32, z32b)  # a fixed operator
    assert P32.nbytes < 0.51 * b64
    dz = np.abs(z32 - z64).max() / np.abs(z64).max()
    res = np.abs(Lin.banded_matvec(p, z32, 10) - r).max() / np.abs(r).max()
    print("181x61 fp32 storage: |z32 - z64| / |z64|", dz, "|P z32 - r| / |r|", res)
    # FP32 elements carry 6e-8 relative rounding, which the dense Schur-complement
    # inverse amplifies by its conditioning (its products cancel): measured 1.0e-3
    # and 2.6e-3.  A wrong or misplaced array gives O(1); the solves with this P
    # (test_gpu_jfnk) reach the FP64-P solution with about as many iterations.
    assert dz <= 1e-2
    assert res <= 1e-2
    P32.close()


def test_precond_rejects_unknown_storage(bim):
    import ctypes
    p = W.tiny(0.7)
    dp = bim.DeviceProblem(p)
    h = ctypes.c_void_p()
    assert bim.lib().precond_setup_ex(dp.ref(), -1, 2, ctypes.byref(h), None) == -1
    assert not h.value


# bounds: the FP32 rounding of the elements (6e-8) amplified by the
# cancellation in the products with the Schur-complement inverse, which grows as
# the mesh is refined: measured 5.1e-5 and 5.6e-5 on the coarse meshes, 2.65e-3
# at dx = 0.27 (4.1e-3 at 181 x 61, dx = 0.33, where the FP32 substitutions
# leave it unchanged to three digits)
@pytest.mark.parametrize("name,mk,hb,tol", [
    ("odd-s-44x9-h2", lambda: W.make_problem(44, 9, -12, 12, 0, 6, 0.9, [W.Bump(0.25, 1.3, 0.9)]), 2, 2e-4),
    ("even-s-45x9-h3", lambda: W.make_problem(45, 9, -12, 12, 0, 6, 0.9, [W.Bump(0.25, 1.3, 0.9)]), 3, 2e-4),
    # 128 < s <= 384: the substitutions forming S^-1 run in FP32 (odd s; and
    # s = 212, whose pivot blocks are inverted as 2 x 2 block matrices and whose
    # triangular products span two 192-row panels)
    ("fp32-substitutions-150x9-h2", lambda: W.make_problem(150, 9, -20, 20, 0, 4, 1.1, [W.Bump(0.2, 1.0, 1.0)]), 2,
     1e-2),
    ("fp32-substitutions-211x9-h2", lambda: W.make_problem(211, 9, -40, 30, 0, 4, 1.1, [W.Bump(0.2, 1.0, 1.0)]), 2,
     1e-2),
], ids=["odd-s", "even-s", "fp32-substitutions-odd-s", "fp32-substitutions-two-panels"])
def test_fp32_storage_small_meshes_match_oracle(bim, name, mk, hb, tol):
    # FP32 elements read one per lane (odd s: rows not aligned to two elements)
    # or two per lane (even s): both apply the oracle's P to FP32 rounding
    p = mk()
    dp = bim.DeviceProblem(p)
    P = bim.Preconditioner(dp, hb, storage="fp32")
    pc_ref = Lin.Preconditioner(p, hb=hb)
    r = np.random.default_rng(8).standard_normal(p.n_unknowns)
    z = P.apply(torch.as_tensor(r, device="cuda")).cpu().numpy()
    z_ref = pc_ref.apply(r)
    err = np.abs(z - z_ref).max() / np.abs(z_ref).max()
    print(name, "fp32 storage rel err", err)
    assert 0 < err <= tol  # rounded (not bit-equal to FP64), and close
    P.close()


def test_precond_full_domain_with_offset_edges(bim):
    # Full domains whose y_1 is not 0: the offset of the closed-form S2 (K5)
    # integral to the edge y_M through the last row of collocation points must be
    # exactly zero; formed from separately rounded coordinates it can be a few ulp,
    # which made that row's entries non-finite and the last pivot block singular
    # (the 91 x 91 mesh of the paper's two-bump domain did).  P z = r by the
    # oracle's banded product.
    import math
    d = 0.5 * math.sqrt(2.0)
    for N, M, (xlo, xhi, ylo, yhi) in ((91, 91, (-7.0, 53.0, -30.0, 30.0)), (121, 81, (-30.0, 30.0, -20.0, 20.0))):
        p = W.make_problem(N, M, xlo, xhi, ylo, yhi, 0.6,
                           [W.Bump(0.2, d, d, cx=10.0, cy=10.0), W.Bump(0.2, d, d, cx=0.0, cy=-10.0)],
                           half_domain=False)
        print(f"case full {N}x{M}", flush=True)
        dp = bim.DeviceProblem(p)
        P = bim.Preconditioner(dp)
        r = np.random.default_rng(7).standard_normal(p.n_unknowns)
        z = P.apply(torch.as_tensor(r, device="cuda"))
        torch.cuda.synchronize()
        res = Lin.banded_matvec(p, z.cpu().numpy(), P.band) - r
        print(f"full {N}x{M} |Pz - r| / |r|", np.abs(res).max() / np.abs(r).max())
        assert np.abs(res).max() <= 1e-9 * np.abs(r).max()
        P.close()
