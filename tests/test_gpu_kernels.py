"""GPU unit checks of single steps of the path, through the kernel-level C entry points:
the contraction GEMM (FP64 and FP32 MFMA), the truncation eigensolve and the Cholesky step of the
QR. Each is compared with a plain float64/complex128 reference of the same operation."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (16, 16, 4), (37, 53, 29), (64, 128, 96), (130, 70, 257)])
@pytest.mark.parametrize("tile", [0, 1])
def test_gemm_fp64(lib, M, N, K, tile):
    print(f"gemm fp64 M={M} N={N} K={K} tile={tile}", flush=True)
    rng = np.random.default_rng(M * 1000 + N + K)
    a, b = crand(rng, M, K), crand(rng, K, N)
    A = torch.from_numpy(a).cuda()
    B = torch.from_numpy(b).cuda()
    C = lib.test_gemm(A, B, acc_fp64=True, tile=tile).cpu().numpy()
    ref = a @ b
    assert np.abs(C - ref).max() <= 1e-13 * np.sqrt(K) * np.abs(a).max() * np.abs(b).max()


@pytest.mark.parametrize("tA,cA,tB,cB", [(1, 1, 0, 0), (0, 0, 1, 1), (1, 0, 1, 0), (0, 1, 0, 1)])
@pytest.mark.parametrize("M,N,K,tile", [(45, 33, 70, 0), (200, 150, 70, 2), (1700, 2100, 37, 1),
                                        (1700, 2100, 37, -1), (300, 270, 45, 3)])
def test_gemm_transpose_conj(lib, tA, cA, tB, cB, M, N, K, tile):
    """Every operand layout (k fastest or not) through both tile sizes of the table-driven kernel
    and the pipelined kernels (64 x 64 with either accumulation; 128 x 128 with FP32, whose FP64
    requests take the 64 x 64 pipeline)."""
    rng = np.random.default_rng(7)
    a = crand(rng, K, M) if tA else crand(rng, M, K)
    b = crand(rng, N, K) if tB else crand(rng, K, N)
    opa = a.T if tA else a
    opb = b.T if tB else b
    opa = opa.conj() if cA else opa
    opb = opb.conj() if cB else opb
    for acc in (True, False):
        dt = torch.complex128 if acc else torch.complex64
        C = lib.test_gemm(torch.from_numpy(a).to(dt).cuda(), torch.from_numpy(b).to(dt).cuda(),
                          transA=bool(tA), conjA=bool(cA), transB=bool(tB), conjB=bool(cB),
                          acc_fp64=acc, tile=tile).cpu().numpy()
        ref = opa @ opb
        tol = 1e-13 if acc else 2e-5
        assert np.abs(C - ref).max() <= tol * np.sqrt(K) * 4, (acc, np.abs(C - ref).max())


@pytest.mark.parametrize("tile", [-1, 0, 1, 2, 3])
@pytest.mark.parametrize("M,N,K", [(32, 32, 16), (100, 200, 300), (257, 65, 64), (64, 64, 16),
                                   (2049, 1793, 100), (4096, 1024, 256)])
def test_gemm_fp32(lib, M, N, K, tile):
    rng = np.random.default_rng(M + N + K)
    a, b = crand(rng, M, K).astype(np.complex64), crand(rng, K, N).astype(np.complex64)
    C = lib.test_gemm(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), acc_fp64=False,
                      tile=tile).cpu().numpy()
    ref = a.astype(np.complex128) @ b.astype(np.complex128)
    assert np.abs(C - ref).max() <= 1e-5 * np.sqrt(K) * 4


@pytest.mark.parametrize("acc", [True, False])
@pytest.mark.parametrize("M,N,K", [(64, 96, 1000), (70, 50, 1500), (256, 1024, 4096), (512, 640, 777)])
def test_gemm_split_k(lib, M, N, K, acc):
    """Few output tiles and a long reduction: the reduction is split into chunks whose sums are added
    in order by a second kernel (the compression's own policy, tile = -1; with FP32 accumulation
    the last two shapes split the pipelined kernel, the first two the table-driven one)."""
    rng = np.random.default_rng(M + N + K)
    dt = np.complex128 if acc else np.complex64
    a, b = crand(rng, M, K).astype(dt), crand(rng, K, N).astype(dt)
    C = lib.test_gemm(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), acc_fp64=acc,
                      tile=-1).cpu().numpy()
    ref = a.astype(np.complex128) @ b.astype(np.complex128)
    tol = 1e-13 if acc else 2e-6
    assert np.abs(C - ref).max() <= tol * np.sqrt(K) * 4 * np.abs(ref).max() / np.sqrt(K), \
        np.abs(C - ref).max()


def herm_psd(rng, s, rank=None, n=None):
    n = n or 2 * s
    m = crand(rng, s, rank or n)
    return m @ m.conj().T


EIG_CASES = [(1, 1), (2, 1), (2, 2), (7, 3), (64, 32), (128, 64), (200, 100), (96, 96), (129, 64),
             (130, 130), (145, 17), (300, 300), (520, 128), (1024, 256), (1100, 64), (1040, 200),
             (1041, 100), (1500, 256), (2064, 64)]


# one-stage sizes: one column before the one-workgroup tail (129) and two (130), the edges of the
# kernel instantiations (columns per thread 1 -> 2 at 512, 2 -> 3 at 1024; rows per workgroup 3 to 7)
MW_CASES = [(129, 64), (130, 130), (200, 100), (300, 300), (512, 100), (513, 256), (700, 200),
            (1024, 256), (1025, 128), (1272, 128), (1300, 64), (1536, 200)]


@pytest.mark.parametrize("s,kmax,reduction",
                         [(s, k, 0) for s, k in EIG_CASES] + [(s, k, 1) for s, k in MW_CASES])
def test_eig_topk(lib, s, kmax, reduction):
    """Top-kmax eigenpairs against numpy.linalg.eigh: the single-workgroup reduction (s <= 128), the
    two-stage reduction (above; panels of up to 1024 and up to 2048 rows, band edges) and, for
    comparison, the one-stage multi-workgroup reduction (third parameter 1)."""
    print(f"eig s={s} kmax={kmax} reduction={reduction}", flush=True)
    rng = np.random.default_rng(s)
    g = herm_psd(rng, s)
    U, lam, kk, inv = lib.test_eig(torch.from_numpy(g).cuda(), kmax, reduction=reduction)
    U = U.cpu().numpy()
    lam = lam.cpu().numpy()
    w, v = np.linalg.eigh(g)
    w, v = w[::-1], v[:, ::-1]
    assert kk == kmax
    assert np.abs(lam - w[:kmax]).max() <= 1e-12 * w[0] * s
    assert abs(inv - 1.0 / np.sqrt(w[0])) <= 1e-12 / np.sqrt(w[0])
    assert np.abs(U.conj().T @ U - np.eye(kmax)).max() <= 1e-12
    # eigen-residual and subspace agreement (projectors compared where a gap exists)
    res = g @ U - U * lam[None, :]
    assert np.abs(res).max() <= 1e-11 * w[0]
    if kmax < s:
        gap = (w[kmax - 1] - w[kmax]) / w[0]
        p_gpu = U @ U.conj().T
        p_ref = v[:, :kmax] @ v[:, :kmax].conj().T
        assert np.abs(p_gpu - p_ref).max() <= 1e-13 / gap * s


def test_eig_multi_workgroup_repeatable(lib):
    """The two-stage reduction (s > 128) sums in a fixed order: repeated solves of the same matrix
    are bitwise identical and match the reference."""
    rng = np.random.default_rng(21)
    s, kmax = 700, 200
    g = herm_psd(rng, s)
    G = torch.from_numpy(g).cuda()
    runs = [lib.test_eig(G, kmax) for _ in range(4)]
    U0, l0 = runs[0][0].cpu().numpy(), runs[0][1].cpu().numpy()
    for U, lam, _, _ in runs[1:]:
        assert np.array_equal(U.cpu().numpy(), U0) and np.array_equal(lam.cpu().numpy(), l0)
    w = np.linalg.eigvalsh(g)[::-1]
    assert np.abs(l0 - w[:kmax]).max() <= 1e-12 * w[0] * s
    assert np.abs(g @ U0 - U0 * l0[None, :]).max() <= 1e-11 * w[0]


def test_eig_multi_workgroup_one_stage_repeatable(lib):
    """The one-stage multi-workgroup reduction (and its one-workgroup tail) sums in a fixed order as
    well: repeated solves are bitwise identical."""
    rng = np.random.default_rng(22)
    s, kmax = 1024, 256
    g = herm_psd(rng, s)
    G = torch.from_numpy(g).cuda()
    runs = [lib.test_eig(G, kmax, reduction=1) for _ in range(3)]
    U0, l0 = runs[0][0].cpu().numpy(), runs[0][1].cpu().numpy()
    for U, lam, _, _ in runs[1:]:
        assert np.array_equal(U.cpu().numpy(), U0) and np.array_equal(lam.cpu().numpy(), l0)
    w = np.linalg.eigvalsh(g)[::-1]
    assert np.abs(l0 - w[:kmax]).max() <= 1e-12 * w[0] * s


@pytest.mark.parametrize("reduction", [0, 1])
def test_eig_rank_deficient_large(lib, reduction):
    """A Gram of rank 300 at s = 700 (the trailing matrix vanishes to rounding long before the
    one-workgroup tail): the top-300 eigenpairs are reproduced and orthonormal. (The vectors of the
    numerically null cluster beyond the rank are not checked: they carry no weight, and the
    Cholesky-QR that follows in a compression drops directions that repeat.)"""
    rng = np.random.default_rng(23)
    s, r, kmax = 700, 300, 400
    g = herm_psd(rng, s, rank=r)
    U, lam, kk, _ = lib.test_eig(torch.from_numpy(g).cuda(), kmax, reduction=reduction)
    U = U.cpu().numpy()
    w = np.linalg.eigvalsh(g)[::-1]
    assert np.abs(lam.cpu().numpy()[:r] - w[:r]).max() <= 1e-11 * w[0]
    p = U[:, :r] @ U[:, :r].conj().T
    assert np.abs(p @ g - g).max() <= 1e-10 * w[0]
    assert np.abs(U[:, :r].conj().T @ U[:, :r] - np.eye(r)).max() <= 1e-11


def test_eig_rank_deficient_and_tol(lib):
    rng = np.random.default_rng(3)
    s, r = 60, 20
    g = herm_psd(rng, s, rank=r)
    U, lam, kk, _ = lib.test_eig(torch.from_numpy(g).cuda(), 40)
    U = U.cpu().numpy()
    w = np.linalg.eigvalsh(g)[::-1]
    assert np.abs(lam.cpu().numpy()[:r] - w[:r]).max() <= 1e-11 * w[0]
    # the top-r subspace is reproduced; the remaining columns span (numerical) null directions
    p = U[:, :r] @ U[:, :r].conj().T
    assert np.abs(p @ g - g).max() <= 1e-10 * w[0]
    # tolerance: keep singular values s_j > tol * s_0  <=>  lam_j > tol^2 lam_0
    tol = np.sqrt(w[9] / w[0]) * 0.999999
    U2, lam2, kk2, _ = lib.test_eig(torch.from_numpy(g).cuda(), 40, tol=tol)
    assert kk2 == 10
    assert np.abs(U2.cpu().numpy()[:, 10:]).max() == 0.0


@pytest.mark.parametrize("s,kind,reduction", [
    (5, "diagonal", 0), (40, "diagonal", 0), (128, "diagonal", 0), (40, "blocks", 0),
    (128, "blocks", 0), (200, "blocks", 0), (300, "diagonal", 0), (333, "blocks", 0),
    (300, "diagonal", 1), (333, "blocks", 1), (1024, "diagonal", 1), (1024, "blocks", 1)])
def test_eig_structured(lib, s, kind, reduction):
    """Grams whose reduction meets columns with nothing below the diagonal (a reflector that is the
    identity, tau = 0): a diagonal Gram (every column) and a block-diagonal one (the last column of
    every block), in the single-workgroup, the two-stage (zero panels and zero band columns) and
    the one-stage multi-workgroup reductions."""
    print(f"eig structured s={s} {kind}", flush=True)
    rng = np.random.default_rng(40 + s)
    if kind == "diagonal":
        g = np.diag(rng.permutation(np.linspace(1.0, 3.0, s))).astype(np.complex128)
    else:
        g = np.zeros((s, s), dtype=np.complex128)
        i0 = 0
        for b in [9, 1, 17, 4, 30, 2, 25, 40, 64, 8]:
            i1 = min(i0 + b, s)
            g[i0:i1, i0:i1] = herm_psd(rng, i1 - i0)
            i0 = i1
            if i0 == s:
                break
        if i0 < s:
            g[i0:, i0:] = herm_psd(rng, s - i0)
    kmax = min(s, 16)
    U, lam, kk, _ = lib.test_eig(torch.from_numpy(g).cuda(), kmax, reduction=reduction)
    U = U.cpu().numpy()
    lam = lam.cpu().numpy()
    w = np.linalg.eigvalsh(g)[::-1]
    assert kk == kmax
    assert np.abs(lam - w[:kmax]).max() <= 1e-12 * w[0] * s
    assert np.abs(U.conj().T @ U - np.eye(kmax)).max() <= 1e-12
    assert np.abs(g @ U - U * lam[None, :]).max() <= 1e-11 * w[0]
    if kind == "diagonal":
        # distinct diagonal entries: the eigenvectors are unit vectors up to a phase
        order = np.argsort(-np.diag(g).real)[:kmax]
        assert np.abs(np.abs(U[order, np.arange(kmax)]) - 1.0).max() <= 1e-12


@pytest.mark.parametrize("s", [50, 260])
def test_eig_degenerate_cluster(lib, s):
    """Exactly repeated eigenvalues: the returned vectors must stay orthonormal."""
    rng = np.random.default_rng(11)
    q, _ = np.linalg.qr(crand(rng, s, s))
    w = np.concatenate([[5.0] * 6, np.linspace(3.0, 0.1, s - 6)])
    g = (q * w) @ q.conj().T
    U, lam, kk, _ = lib.test_eig(torch.from_numpy(g).cuda(), 10)
    U = U.cpu().numpy()
    assert np.abs(U.conj().T @ U - np.eye(10)).max() <= 1e-11
    assert np.abs(g @ U - U * lam.cpu().numpy()[None, :]).max() <= 1e-11 * 5


@pytest.mark.parametrize("k", [1, 5, 64, 88, 89, 130, 256, 300])
def test_chol_inv(lib, k):
    """LDS-resident sizes (k <= 88) and the blocked factorisation above them."""
    rng = np.random.default_rng(k)
    g = herm_psd(rng, k)
    Ci, nd = lib.test_chol_inv(torch.from_numpy(g).cuda())
    Ci = Ci.cpu().numpy()
    assert nd == 0
    c = np.linalg.cholesky(g)
    assert np.abs(Ci - np.linalg.inv(c)).max() <= 1e-10 * np.abs(np.linalg.inv(c)).max()
    assert np.abs(np.triu(Ci, 1)).max() == 0.0


@pytest.mark.parametrize("k", [64, 200])
@pytest.mark.parametrize("eps", [1e-16, 1e-9])
def test_chol_inv_near_identity(lib, eps, k):
    """A re-orthogonalisation pass (no shift) on a Gram within rounding of the identity returns the
    identity; a larger deviation is factorised as usual. Both are the inverse Cholesky factor to
    rounding. k = 200 takes the blocked factorisation, whose steps all stand down after the
    identity check."""
    rng = np.random.default_rng(5)
    e = crand(rng, k, k) * eps
    g = np.eye(k) + (e + e.conj().T) / 2
    Ci, nd = lib.test_chol_inv(torch.from_numpy(g).cuda())
    Ci = Ci.cpu().numpy()
    ref = np.linalg.inv(np.linalg.cholesky(g))
    assert nd == 0
    assert np.abs(Ci - ref).max() <= 1e-13
    if eps < 1e-15:
        assert np.array_equal(Ci, np.eye(k))


@pytest.mark.parametrize("k,r", [(24, 15), (200, 130)])
def test_chol_inv_drops_zero_pivots(lib, k, r):
    rng = np.random.default_rng(2)
    s = crand(rng, r, max(40, 2 * r))
    s = np.concatenate([s, np.zeros((k - r, s.shape[1]))])
    perm = rng.permutation(k)
    s = s[perm]
    g = s @ s.conj().T
    Ci, nd = lib.test_chol_inv(torch.from_numpy(g).cuda(), drop_rel=1e-13)
    Ci = Ci.cpu().numpy()
    assert nd == k - r
    q = Ci @ s
    nz = np.abs(q).sum(axis=1) > 0
    assert nz.sum() == r
    qq = q[nz]
    assert np.abs(qq @ qq.conj().T - np.eye(r)).max() <= 1e-10
