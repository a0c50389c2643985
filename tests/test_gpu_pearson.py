"""The co-expression prior on the GPU (Sec. II-A: Pearson correlation between
genes across samples, panda_pearson) against the FP64 oracle from the same
FP32 expression matrix: every entry at small and ragged sizes, sampled
entries at the realistic size (18000 genes x 200 samples)."""
import ctypes as ct

import numpy as np
import pytest

from paper_1507_07039_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-5  # |r| <= 1; FP32 product of unit-norm rows over <= 320 samples


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def pd(torch):
    from paper_1507_07039_amd import panda
    panda.load_library()
    return panda


def gpu_pearson(torch, pd, E32, pad=0):
    """panda_pearson through the C ABI, E with leading dimension S + pad."""
    G, S = E32.shape
    buf = np.zeros((G, S + pad), np.float32)
    buf[:, :S] = E32
    Ed = torch.from_numpy(buf).cuda()
    Cd = torch.full((G, G + 3), float("nan"), dtype=torch.float32, device="cuda")
    lib = pd.load_library()
    ws = pd.workspace(lib.panda_pearson_workspace_bytes(G, S))
    st = lib.panda_pearson(ct.c_void_p(Ed.data_ptr()), G, S, S + pad, ct.c_void_p(Cd.data_ptr()),
                           G + 3, ct.c_void_p(ws.data_ptr()), ws.numel(), pd._stream())
    assert st == pd.OK, lib.panda_last_error()
    torch.cuda.synchronize()
    C = Cd.cpu().numpy()
    assert np.all(np.isnan(C[:, G:])), "wrote past the G columns of a row"
    return C[:, :G]


@pytest.mark.parametrize("G,S,pad", [(400, 30, 0), (333, 37, 5), (129, 2, 0), (1, 7, 0),
                                     (700, 300, 3)])
def test_full_matrix_matches_oracle(torch, pd, oracle, G, S, pad):
    rng = np.random.default_rng(G * 1000 + S)
    if (G, S) == (400, 30):
        E = I.workload_expression(I.SMALL)
    else:
        E = rng.normal(size=(G, S)) * rng.uniform(0.1, 30.0, size=(G, 1)) + rng.normal(size=(G, 1))
    E32 = E.astype(np.float32)
    if G > 10:  # constant rows: zero and non-zero level
        E32[3] = 0.0
        E32[G - 1] = 4.25
    C = gpu_pearson(torch, pd, E32, pad)
    ref = oracle.pearson(E32.astype(np.float64))
    err = np.abs(C.astype(np.float64) - ref).max()
    print(f"G={G} S={S} lde={S + pad}: max|C - oracle| {err:.2e}")
    assert err <= TOL
    assert np.all(np.diag(C) == 1.0)
    if G > 10:
        for r in (3, G - 1):
            assert np.all(np.delete(C[r], r) == 0.0) and np.all(np.delete(C[:, r], r) == 0.0)


def test_realistic_size_sampled(torch, pd, oracle):
    """18000 genes x 200 samples (the expression of the T=700, G=18000
    workload): 20000 random entries, one full row and the diagonal against
    the oracle; the whole matrix symmetric to FP32 rounding; its z-score
    equal to the z-scored C0 the message-passing tests start from."""
    E = I.workload_expression(I.HUMAN)
    E32 = E.astype(np.float32)
    G = E32.shape[0]
    Ed = torch.from_numpy(E32).cuda()
    C = pd.pearson(Ed)
    torch.cuda.synchronize()
    rng = np.random.default_rng(18000)
    r = np.concatenate([rng.integers(0, G, 20000), np.full(G, 4321), np.arange(G)])
    c = np.concatenate([rng.integers(0, G, 20000), np.arange(G), np.arange(G)])
    ref = oracle.pearson_entries(E32.astype(np.float64), r, c)
    got = C[torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda()].cpu().numpy().astype(np.float64)
    err = np.abs(got - ref).max()
    asym = (C - C.T).abs().max().item()
    print(f"G={G} S={E32.shape[1]}: max|C - oracle| over {r.size} entries {err:.2e}, "
          f"max|C - C^T| {asym:.2e}")
    assert err <= TOL and asym <= 1e-6
    # the prior as the message passing receives it: z-scored on the GPU
    pd.normalize(C)
    _, _, C0 = I.workload_priors(I.HUMAN)
    z0 = oracle.normalize(C0)
    zerr = np.abs(C[torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda()].cpu().numpy() - z0[r, c]).max()
    print(f"z-scored: max|C - oracle| {zerr:.2e}")
    assert zerr <= 1e-3
    del C


def test_timing(torch, pd):
    """Time of the front end at the realistic size (printed; the JSON driver
    is paper_1507_07039_amd.prior)."""
    from paper_1507_07039_amd import prior
    res = prior.measure(18000, 200, reps=5, torch=torch, panda=pd)
    print(res)
    assert res["ms"] > 0 and res["roofline"]["frac"] > 0
