"""GPU checks of the building blocks through the C interface: the MFMA
matrix products (FP64, FP32, BF16 with FP32 accumulation; all operand
layouts, batches, split-K, ragged tiles) and the blocked Householder QR."""
import numpy as np
import pytest
import torch

from paper_2509_05090_amd import ctm

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")
TDT = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16}


def _rng(seed):
    return np.random.default_rng(seed)


def _stored(x, prec):
    """Host copy of the values a device operand of type prec actually holds."""
    return torch.tensor(x).to(TDT[prec]).double().numpy()


def run_gemm(M, N, K, prec, ta, tb, seed, ksplit=0, alpha=1.0, beta=0.0, ctype=None):
    r = _rng(seed)
    ctype = prec if ctype is None else ctype
    A = r.standard_normal((K, M) if ta else (M, K))
    B = r.standard_normal((N, K) if tb else (K, N))
    C0 = r.standard_normal((M, N))
    Ad = torch.tensor(A, device=DEV).to(TDT[prec])
    Bd = torch.tensor(B, device=DEV).to(TDT[prec])
    Cd = torch.tensor(C0, device=DEV).to(TDT[ctype])
    ctm.gemm(Ad, Bd, Cd, M, N, K, lda=M if ta else K, ldb=K if tb else N, ldc=N, transA=ta,
             transB=tb, alpha=alpha, beta=beta, prec=prec, ksplit=ksplit)
    torch.cuda.synchronize()
    Ah, Bh = _stored(A, prec), _stored(B, prec)
    opA = Ah.T if ta else Ah
    opB = Bh.T if tb else Bh
    ref = alpha * opA @ opB + beta * _stored(C0, ctype)
    scale = alpha * np.abs(opA) @ np.abs(opB) + abs(beta) * np.abs(C0) + 1e-300
    err = np.abs(Cd.double().cpu().numpy() - ref) / scale
    return err.max()


TOL = {0: 1e-14, 1: 2e-6, 2: 2e-6}
TOL_OUT = {0: 1e-14, 1: 2e-6, 2: 5e-3}  # output stored in the operand type


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 5, 3), (100, 37, 45), (130, 144, 300),
                                   (64, 48, 129), (33, 200, 1000)])
def test_gemm_layouts(prec, ta, tb, M, N, K):
    seed = M * 7919 + N * 31 + K + prec * 1000003 + 2 * ta + tb
    err = run_gemm(M, N, K, prec, ta, tb, seed)
    # no split and same output type -> output rounded to the operand type
    assert err < max(TOL[prec], TOL_OUT[prec]), err


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_gemm_split_k_fp64_output(prec):
    err = run_gemm(70, 48, 5000, prec, False, False, 11, ksplit=7, ctype=0)
    assert err < TOL[prec] * 10, err
    err = run_gemm(300, 144, 5184, prec, False, True, 12, ksplit=0, ctype=0)
    assert err < TOL[prec] * 10, err


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
@pytest.mark.parametrize("M,N,K,ksplit", [(136, 40, 264, 0), (134, 45, 261, 0), (70, 150, 1029, 3),
                                          (200, 144, 5000, 0)])
def test_gemm_aligned_operands(prec, ta, tb, M, N, K, ksplit):
    """Leading dimensions padded to multiples of 16 bytes, so the 16-byte
    load path runs, with ragged tiles and partial vectors at the k and m/n
    ends (K, M, N not multiples of the vector width)."""
    r = _rng(M * 31 + N * 7 + K + prec * 101 + 4 * ta + 2 * tb + ksplit)
    pad = lambda x: (x + 7) // 8 * 8
    ra, ca = (K, M) if ta else (M, K)
    rb, cb = (N, K) if tb else (K, N)
    A = r.standard_normal((ra, pad(ca)))
    B = r.standard_normal((rb, pad(cb)))
    Ad = torch.tensor(A, device=DEV).to(TDT[prec])
    Bd = torch.tensor(B, device=DEV).to(TDT[prec])
    Cd = torch.zeros((M, N), device=DEV, dtype=torch.float64)
    ctm.gemm(Ad, Bd, Cd, M, N, K, lda=pad(ca), ldb=pad(cb), ldc=N, transA=ta, transB=tb,
             prec=prec, ksplit=ksplit)
    torch.cuda.synchronize()
    Ah, Bh = _stored(A, prec)[:, :ca], _stored(B, prec)[:, :cb]
    opA = Ah.T if ta else Ah
    opB = Bh.T if tb else Bh
    ref = opA @ opB
    scale = np.abs(opA) @ np.abs(opB) + 1e-300
    err = (np.abs(Cd.cpu().numpy() - ref) / scale).max()
    assert err < TOL[prec] * 10, err


def test_gemm_alpha_beta_in_place():
    err = run_gemm(200, 100, 16, 0, False, False, 13, ksplit=1, alpha=-1.0, beta=1.0)
    assert err < 1e-14


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_gemm_two_level_batch(prec):
    """C[b0][b1] = A[b0] B[b1] with independent strides, ragged 36-wide tiles."""
    r = _rng(21)
    nb0, nb1, M, N, K = 3, 4, 40, 36, 36
    A = r.standard_normal((nb0, K, M))        # transposed operand, batched over b0
    B = r.standard_normal((nb1, K, N))        # batched over b1
    Ad = torch.tensor(A, device=DEV).to(TDT[prec])
    Bd = torch.tensor(B, device=DEV).to(TDT[prec])
    Cd = torch.zeros((nb0, nb1, M, N), device=DEV, dtype=TDT[prec])
    ctm.gemm(Ad, Bd, Cd, M, N, K, lda=M, ldb=N, ldc=N, transA=True, prec=prec, batch=(nb0, nb1),
             sA=(K * M, 0), sB=(0, K * N), sC=(nb1 * M * N, M * N))
    torch.cuda.synchronize()
    Ah, Bh = _stored(A, prec), _stored(B, prec)
    ref = np.einsum("akm,bkn->abmn", Ah, Bh)
    scale = np.einsum("akm,bkn->abmn", np.abs(Ah), np.abs(Bh))
    err = np.abs(Cd.double().cpu().numpy() - ref) / scale
    assert err.max() < max(TOL[prec], TOL_OUT[prec]), err.max()


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("nb0,nb1,M,N,K,ta,tb", [(5, 7, 144, 36, 36, True, False),
                                                  (3, 4, 256, 64, 64, True, False),
                                                  (4, 3, 100, 20, 50, False, True),
                                                  (2, 5, 17, 64, 3, False, False),
                                                  (3, 2, 40, 9, 64, True, True),
                                                  (1, 5, 200, 144, 36, False, False),
                                                  (2, 3, 70, 100, 30, True, False)])
def test_gemm_small_batches(prec, nb0, nb1, M, N, K, ta, tb):
    """Batched products with small K and A shared across the second batch
    index (the pair contractions of the enlarged corner), several row tiles
    of A, both operand layouts; C[b0][b1] lives in a padded row layout.
    K, N <= 64 takes the small-batch kernel, the N > 64 cases the general
    batched one."""
    r = _rng(nb0 * 1009 + nb1 * 101 + M + N + K + prec + 2 * ta + tb)
    A = r.standard_normal((nb0,) + ((K, M) if ta else (M, K)))
    B = r.standard_normal((nb1,) + ((N, K) if tb else (K, N)))
    ldc = N + 3
    Ad = torch.tensor(A, device=DEV).to(TDT[prec])
    Bd = torch.tensor(B, device=DEV).to(TDT[prec])
    Cd = torch.full((nb0, nb1, M, ldc), 7.0, device=DEV, dtype=TDT[prec])
    ctm.gemm(Ad, Bd, Cd, M, N, K, lda=M if ta else K, ldb=K if tb else N, ldc=ldc, transA=ta,
             transB=tb, prec=prec, batch=(nb0, nb1), sA=(K * M, 0), sB=(0, K * N),
             sC=(nb1 * M * ldc, M * ldc))
    torch.cuda.synchronize()
    Ah, Bh = _stored(A, prec), _stored(B, prec)
    opA = np.swapaxes(Ah, 1, 2) if ta else Ah
    opB = np.swapaxes(Bh, 1, 2) if tb else Bh
    ref = np.einsum("amk,bkn->abmn", opA, opB)
    scale = np.einsum("amk,bkn->abmn", np.abs(opA), np.abs(opB)) + 1e-300
    out = Cd.double().cpu().numpy()
    err = (np.abs(out[..., :N] - ref) / scale).max()
    assert err < max(TOL[prec], TOL_OUT[prec]), err
    assert np.all(out[..., N:] == 7.0)  # padding columns untouched


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("nb0,nb1,M,N,K,tb,ldc", [(5, 7, 144, 36, 36, False, 40),
                                                   (17, 9, 36, 36, 36, True, 36),
                                                   (3, 4, 20, 16, 16, False, 20),
                                                   (2, 5, 64, 64, 64, True, 64),
                                                   (4, 3, 8, 4, 4, False, 8),
                                                   (3, 2, 52, 20, 50, True, 24)])
def test_gemm_small_batches_row_layout(prec, nb0, nb1, M, N, K, tb, ldc):
    """Small batches with A stored rows-contiguous and output rows of whole
    4-element groups (the layout of the enlarged-corner pair contractions):
    every (K, N) instance size, 16-row tiles with a ragged last tile, a last
    group of b0 batches and of b1 batches only partly filled, both layouts
    of B; the padding columns of C stay untouched."""
    r = _rng(nb0 * 2003 + nb1 * 31 + M + N + K + prec + tb)
    A = r.standard_normal((nb0, K, M))
    B = r.standard_normal((nb1,) + ((N, K) if tb else (K, N)))
    Ad = torch.tensor(A, device=DEV).to(TDT[prec])
    Bd = torch.tensor(B, device=DEV).to(TDT[prec])
    Cd = torch.full((nb0, nb1, M, ldc), 7.0, device=DEV, dtype=TDT[prec])
    ctm.gemm(Ad, Bd, Cd, M, N, K, lda=M, ldb=K if tb else N, ldc=ldc, transA=True, transB=tb,
             prec=prec, batch=(nb0, nb1), sA=(K * M, 0), sB=(0, K * N),
             sC=(nb1 * M * ldc, M * ldc))
    torch.cuda.synchronize()
    Ah, Bh = _stored(A, prec), _stored(B, prec)
    opB = np.swapaxes(Bh, 1, 2) if tb else Bh
    ref = np.einsum("akm,bkn->abmn", Ah, opB)
    scale = np.einsum("akm,bkn->abmn", np.abs(Ah), np.abs(opB)) + 1e-300
    out = Cd.double().cpu().numpy()
    err = (np.abs(out[..., :N] - ref) / scale).max()
    assert err < max(TOL[prec], TOL_OUT[prec]), err
    assert np.all(out[..., N:] == 7.0)


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("nb0,M", [(20, 44), (9, 144)])
def test_gemm_small_batches_v3_layout(prec, nb0, M):
    """The V3 product's output layout: C[(b1, row)][(b0, col)], so the
    results of consecutive b0 batches sit side by side in one output row
    (N = K = 36, B read transposed)."""
    nb1, N, K = 36, 36, 36
    r = _rng(nb0 * 7 + M + prec)
    A = r.standard_normal((nb0, K, M))
    B = r.standard_normal((N, nb1, K))  # B[b1](k, n) = a[n][b1][k]
    Ad = torch.tensor(A, device=DEV).to(TDT[prec])
    Bd = torch.tensor(B, device=DEV).to(TDT[prec])
    Cd = torch.zeros((nb1, M, nb0, N), device=DEV, dtype=TDT[prec])
    ctm.gemm(Ad, Bd, Cd, M, N, K, lda=M, ldb=nb1 * K, ldc=nb0 * N, transA=True, transB=True,
             prec=prec, batch=(nb0, nb1), sA=(K * M, 0), sB=(0, K), sC=(N, M * nb0 * N))
    torch.cuda.synchronize()
    Ah, Bh = _stored(A, prec), _stored(B, prec)
    ref = np.einsum("akm,nbk->bman", Ah, Bh)
    scale = np.einsum("akm,nbk->bman", np.abs(Ah), np.abs(Bh)) + 1e-300
    err = (np.abs(Cd.double().cpu().numpy() - ref) / scale).max()
    assert err < max(TOL[prec], TOL_OUT[prec]), err


QR_SHAPES = [(16, 16), (40, 16), (200, 37), (1024, 64), (1600, 100), (5184, 144), (144, 144),
             (513, 33), (1025, 64), (9000, 100), (16384, 256), (30000, 40), (7, 1),
             (512, 40), (8192, 64)]


@pytest.mark.parametrize("n,k", QR_SHAPES)
def test_householder_qr(n, k):
    """Shapes with one leaf, several leaves (ragged last leaf), two rows per
    thread in the leaves (n > 8192) and in the stacked factorization; leaves
    and stacked rows at the 512 (32-column panels) and 1024 (16-column)
    rows a workgroup holds (512 x 40, 8192 x 64, 16384 x 256)."""
    M = _rng(n + k).standard_normal((n, k))
    Q, R = ctm.qr(torch.tensor(M, device=DEV))
    torch.cuda.synchronize()
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    assert np.abs(np.tril(R, -1)).max() == 0.0
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 1e-13
    assert np.abs(Q @ R - M).max() < 1e-13 * np.abs(M).max() * np.sqrt(n)
    # same triangular factor as LAPACK up to row signs, LAPACK's sign convention
    Rl = np.linalg.qr(M, mode="r")
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rl)), rtol=1e-12)


def test_householder_qr_rank_deficient():
    """A matrix of rank 1 (the product-state case) must still give an
    orthonormal Q and Q R = M."""
    r = _rng(5)
    u, v = r.standard_normal((300, 1)), r.standard_normal((1, 20))
    M = u @ v
    Q, R = ctm.qr(torch.tensor(M, device=DEV))
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    assert np.abs(Q.T @ Q - np.eye(20)).max() < 1e-13
    assert np.abs(Q @ R - M).max() < 1e-12 * np.abs(M).max()


def test_householder_qr_ill_conditioned():
    """Columns scaled over 12 decades (the reduced corner's spread): Q must
    stay orthonormal and span the same space as LAPACK's Q column by column
    (the leading j columns of both span the same space)."""
    r = _rng(9)
    n, k = 5184, 144
    M = r.standard_normal((n, k)) * np.logspace(0, -12, k)[None, :]
    Q, R = ctm.qr(torch.tensor(M, device=DEV))
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 1e-13
    assert np.abs(Q @ R - M).max() < 1e-13 * np.abs(M).max() * np.sqrt(n)
    Ql, _ = np.linalg.qr(M)
    # column j of Q equals +-column j of LAPACK's Q up to the conditioning of
    # the leading j columns; compare the projectors on the first 20 columns
    P1, P2 = Q[:, :20] @ Q[:, :20].T, Ql[:, :20] @ Ql[:, :20].T
    assert np.abs(P1 - P2).max() < 1e-9


def test_householder_qr_repeated_calls_are_identical():
    """The stacked factorization is done by whichever leaf finishes last;
    results must not depend on that order."""
    M = torch.tensor(_rng(77).standard_normal((5184, 144)), device=DEV)
    Q1, R1 = ctm.qr(M)
    for _ in range(3):
        Q2, R2 = ctm.qr(M)
        assert torch.equal(Q1, Q2) and torch.equal(R1, R2)
