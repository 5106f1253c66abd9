"""Factor build through the integer Gram (int8 digit products, the default for
FP32 / FP16 / BF16 / matrix-free storage) against the FP64-instruction Gram
of the same stored operator, and against a CPU FP64 inverse of the exact
stored values.

Shapes exercise the edge cases of the integer path: KM = 96 rows (the last
64-row tile half empty), N = 8464 pixels (two 8192-column chunks, the
second ragged), N = 16900 (three chunks), a compacted operator after
pruning.

Tolerance.  The integer path rounds each entry to 30 bits below its row's
largest magnitude and drops digit pairs of weight <= 2^-40; an exact CPU
emulation of that arithmetic on the N = 8464 problem gives a Gram
error of ~4e-12 relative to its largest entry and a factor error of ~2e-9
(Frobenius, relative), the condition number of rho I + G being ~1.4e4.  The
bar 1e-7 leaves a factor 50; dropping the s + t = 4 pairs (error 9e-6)
fails it.
"""

import numpy as np
import pytest

from scenegen import make_geometry, steering

pytestmark = pytest.mark.gpu


def _factors(lib, g, A, y, storage, gram, mask=None):
    s = lib.Solver(g.Q, g.K, g.M, g.N, storage=storage, gram=gram, lam=0.05, max_iter=1,
                   stop=False, reuse_factor=False)
    for q in range(g.Q):
        if storage == "mf":
            s.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
        else:
            s.set_operator(q, A[q])
        if mask is not None:
            s.set_active_mask(q, mask[q])
    s.solve(y)
    W = [s.factor(q) for q in range(g.Q)]
    s.close()
    return W


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def problem():
    g = make_geometry(2, 3, 32, 92)          # KM = 96, N = 8464
    A = [steering(g, q).astype(np.complex64) for q in range(g.Q)]
    rng = np.random.default_rng(5)
    y = (rng.standard_normal((g.Q, g.K * g.M)) + 1j * rng.standard_normal((g.Q, g.K * g.M)))
    return g, A, y.astype(np.complex64)


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16", "mf"])
def test_integer_gram_factor_matches_fp64_gram(gpu_lib, problem, storage):
    g, A, y = problem
    Wi = _factors(gpu_lib, g, A, y, storage, "int8")
    Wd = _factors(gpu_lib, g, A, y, storage, "fp64")
    for q in range(g.Q):
        err = _rel(Wi[q], Wd[q])
        print(storage, q, f"{err:.3e}")
        assert err <= 1e-7, (storage, q, err)
        assert np.allclose(Wi[q], Wi[q].conj().T, rtol=0, atol=1e-14 * np.abs(Wi[q]).max())


def test_integer_gram_factor_matches_cpu_inverse(gpu_lib, problem):
    """FP32 storage holds exactly A.astype(complex64): the CPU FP64 factor of
    those values is the reference of both Gram paths."""
    g, A, y = problem
    rho = 2.0                                  # (beta + gamma) / mu
    Wi = _factors(gpu_lib, g, A, y, "fp32", "int8")
    Wd = _factors(gpu_lib, g, A, y, "fp32", "fp64")
    for q in range(g.Q):
        Aq = A[q].astype(np.complex128)
        Wref = np.linalg.inv(rho * np.eye(Aq.shape[0]) + Aq @ Aq.conj().T)
        ei, ed = _rel(Wi[q], Wref), _rel(Wd[q], Wref)
        print(q, f"int8 {ei:.3e}  fp64 {ed:.3e}")
        assert ed <= 1e-10
        assert ei <= 1e-7


def test_integer_gram_on_compacted_operator(gpu_lib, problem):
    """A caller selector leaves a ragged active set (columns gathered before
    the Gram): both paths agree on the factor of the compacted operator."""
    g, A, y = problem
    rng = np.random.default_rng(9)
    mask = [(rng.random(g.N) < 0.37).astype(np.uint8) for _ in range(g.Q)]
    Wi = _factors(gpu_lib, g, A, y, "fp32", "int8", mask)
    Wd = _factors(gpu_lib, g, A, y, "fp32", "fp64", mask)
    rho = 2.0
    for q in range(g.Q):
        Aq = A[q][:, mask[q].astype(bool)].astype(np.complex128)
        Wref = np.linalg.inv(rho * np.eye(Aq.shape[0]) + Aq @ Aq.conj().T)
        assert _rel(Wd[q], Wref) <= 1e-10
        assert _rel(Wi[q], Wref) <= 1e-7


@pytest.mark.parametrize("storage", ["fp32", "mf"])
def test_integer_gram_three_chunks_matches_fp64_gram(gpu_lib, storage):
    """N = 16900: the integer products run as three column chunks (the third
    adds 516 columns).  Same 1e-7 bar against the FP64-Gram factor of the
    same stored operator."""
    g = make_geometry(2, 3, 32, 130)         # KM = 96, N = 16900
    A = [steering(g, q).astype(np.complex64) for q in range(g.Q)]
    rng = np.random.default_rng(6)
    y = (rng.standard_normal((g.Q, g.K * g.M)) + 1j * rng.standard_normal((g.Q, g.K * g.M)))
    y = y.astype(np.complex64)
    Wi = _factors(gpu_lib, g, A, y, storage, "int8")
    Wd = _factors(gpu_lib, g, A, y, storage, "fp64")
    for q in range(g.Q):
        err = _rel(Wi[q], Wd[q])
        print(storage, q, f"{err:.3e}")
        assert err <= 1e-7, (storage, q, err)


@pytest.mark.parametrize("shape", [(2, 3, 32, 92), (3, 4, 40, 60), (2, 8, 128, 40)])
def test_wide_and_narrow_instruction_grams_are_identical(gpu_lib, shape):
    """The integer Gram on the 16x16x64 instruction (default) and on the
    32x32x32 one sum the same int8 digit products into the same int32 class
    accumulators, so the factors are equal bit for bit: KM = 96 (half-empty
    last row tile), N = 8464 (two chunks, the second ragged); KM = 160,
    N = 3600; KM = 1024 (16 row tiles, 136 tiles per sensor), N = 1600."""
    Q, M, K, n_side = shape
    g = make_geometry(Q, M, K, n_side)
    A = [steering(g, q).astype(np.complex64) for q in range(g.Q)]
    rng = np.random.default_rng(7)
    y = (rng.standard_normal((g.Q, g.K * g.M)) + 1j * rng.standard_normal((g.Q, g.K * g.M)))
    y = y.astype(np.complex64)
    for storage in ("fp32", "bf16"):
        Wn = _factors(gpu_lib, g, A, y, storage, "int8")
        Ww = _factors(gpu_lib, g, A, y, storage, "int8_32")
        for q in range(g.Q):
            assert np.array_equal(Ww[q], Wn[q]), (storage, q)


def test_shared_workspace_across_handles_and_streams(gpu_lib, problem):
    """The digit-plane workspace is one per device: handles on two streams
    building factors back to back (each build ordered after the previous
    user's Gram kernels by an event) get the factors of a handle alone."""
    import torch
    g, A, y = problem
    ref = _factors(gpu_lib, g, A, y, "fp32", "int8")
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    hs = []
    for st in streams:
        s = gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", lam=0.05, max_iter=1, stop=False,
                           reuse_factor=False, stream=st.cuda_stream)
        for q in range(g.Q):
            s.set_operator(q, A[q])
        hs.append(s)
    for _ in range(2):
        for s in hs:
            s.solve(y)
    torch.cuda.synchronize()
    for s in hs:
        for q in range(g.Q):
            assert np.array_equal(s.factor(q), ref[q])
        s.close()
