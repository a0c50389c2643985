"""The permutation null on the GPU (node-label randomisation, Sec. III;
panda_permute_sym, panda_null, panda_null_zscore) against the FP64 oracle:
relabelling bit for bit, null mean and sd of small networks element by
element, identity relabellings reproducing the plain run exactly, and at the
T=700, G=18000 size a relabelled instance against the plain run of the
relabelled motif prior."""
import ctypes as ct

import numpy as np
import pytest

from oracle import null as N
from paper_1507_07039_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-4  # per-run W bound of the FP32 path; mean and sd are 1-Lipschitz in it


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


def f32(oracle, *Ms):
    return tuple(np.ascontiguousarray(oracle.normalize(M).astype(np.float32)) for M in Ms)


def dev(torch, *arrs):
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs)


def perms(seed, K, n):
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(n) for _ in range(K)]).astype(np.int32)


@pytest.mark.parametrize("n", [1, 7, 400, 1000])
def test_permute_sym_exact(torch, pd, n):
    rng = np.random.default_rng(n)
    M = rng.normal(size=(n, n)).astype(np.float32)
    p = rng.permutation(n).astype(np.int32)
    (Md, pdv) = dev(torch, M, p)
    out = pd.permute_sym(Md, pdv).cpu().numpy()
    assert np.array_equal(out, N.permute_sym(M, p).astype(np.float32))


@pytest.mark.parametrize("n", [40960, 40961])
def test_permute_sym_row_staging_limit(torch, pd, n):
    """Both sides of the largest row the kernel stages in LDS (160 KB = 40960
    floats; longer rows take the kernel that gathers from global memory):
    bit for bit against torch's own indexing of the same device matrix."""
    g = torch.Generator(device="cuda").manual_seed(n)
    M = torch.randn((n, n), generator=g, device="cuda", dtype=torch.float32)
    p = torch.randperm(n, generator=g, device="cuda").to(torch.int32)
    out = pd.permute_sym(M, p)
    pl = p.long()
    want = M.index_select(0, pl).index_select(1, pl)
    assert torch.equal(out, want)
    del M, out, want
    torch.cuda.empty_cache()


def test_permute_sym_rejects_non_permutations(torch, pd):
    lib = pd.load_library()
    M = torch.zeros((5, 5), dtype=torch.float32, device="cuda")
    out = torch.zeros((5, 5), dtype=torch.float32, device="cuda")
    for bad in ([0, 1, 2, 3, 3], [0, 1, 2, 3, 5], [-1, 0, 1, 2, 3]):
        p = torch.tensor(bad, dtype=torch.int32, device="cuda")
        st = lib.panda_permute_sym(ct.c_void_p(M.data_ptr()), 5, 5, ct.c_void_p(p.data_ptr()),
                                   ct.c_void_p(out.data_ptr()), 5, pd._stream())
        assert st == pd.ERR_ARG, bad
    assert torch.count_nonzero(out).item() == 0


@pytest.mark.parametrize("case", ["genes", "genes+tfs"])
def test_null_matches_oracle(torch, pd, oracle, case):
    if case == "genes":
        W, P, C = f32(oracle, *I.workload_priors(I.SMALL))
        K, gp, tp = 4, perms(11, 4, 400), None
    else:  # ragged sizes, both priors relabelled
        W, P, C = f32(oracle, *I.priors(257, 33, 257, 0.05, 0.03, 30, 8))
        K, gp, tp = 3, perms(12, 3, 257), perms(13, 3, 33)
    mean_o, sd_o, it_o, _ = N.null_stats(*(a.astype(np.float64) for a in (W, P, C)),
                                         gene_perms=gp, tf_perms=tp)
    Wd, Pd, Cd = dev(torch, W, P, C)
    res = pd.null(Wd, Pd, Cd, gene_perm=dev(torch, gp)[0],
                  tf_perm=None if tp is None else dev(torch, tp)[0])
    torch.cuda.synchronize()
    em = np.abs(res.mean.cpu().numpy().astype(np.float64) - mean_o).max()
    es = np.abs(res.sd.cpu().numpy().astype(np.float64) - sd_o).max()
    print(f"{case}: K={K} iterations gpu {res.iters} oracle {it_o}; max|mean - oracle| {em:.2e}, "
          f"max|sd - oracle| {es:.2e}, max sd {sd_o.max():.3f}")
    assert res.status == pd.OK and res.iters == it_o
    assert em <= TOL and es <= TOL
    # z-scores of the real network against the null
    real = pd.run(Wd, Pd, Cd)
    z = pd.null_zscore(real.W, res.mean, res.sd).cpu().numpy()
    zo = N.zscore(real.W.cpu().numpy(), res.mean.cpu().numpy(), res.sd.cpu().numpy())
    assert np.abs(z - zo).max() <= 1e-5 * max(1.0, np.abs(zo).max())


def test_identity_relabelling_is_the_plain_run(torch, pd, oracle):
    W, P, C = f32(oracle, *I.workload_priors(I.SMALL))
    Wd, Pd, Cd = dev(torch, W, P, C)
    ident = torch.arange(400, dtype=torch.int32, device="cuda").repeat(3, 1).contiguous()
    res = pd.null(Wd, Pd, Cd, gene_perm=ident)
    real = pd.run(Wd, Pd, Cd)
    torch.cuda.synchronize()
    assert torch.equal(res.mean, real.W)
    assert torch.count_nonzero(res.sd).item() == 0
    assert res.iters == [real.iters] * 3


def test_realistic_size_relabelled_instance(torch, pd, oracle):
    """T=700, G=18000, three iterations (tol 0): one null instance with its
    genes relabelled by s equals the plain run of W0[:, s^-1] read back as
    [:, s], to FP32 rounding; the relabelled C is exact on sampled entries."""
    W0, P0, C0 = I.workload_priors(I.HUMAN)
    W, P, C = f32(oracle, W0, P0, C0)
    del W0, P0, C0
    Ne, Na = W.shape
    s = perms(18000, 1, Na)
    inv = np.empty_like(s[0])
    inv[s[0]] = np.arange(Na, dtype=np.int32)
    Wd, Pd, Cd, sd_ = dev(torch, W, P, C, s)
    Cp = pd.permute_sym(Cd, sd_[0].contiguous())
    rng = np.random.default_rng(5)
    r, c = rng.integers(0, Na, 20000), rng.integers(0, Na, 20000)
    got = Cp[torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda()].cpu().numpy()
    assert np.array_equal(got, C[s[0][r], s[0][c]])
    del Cp
    o = pd.default_options(tol=0.0, max_iter=3)
    res = pd.null(Wd, Pd, Cd, gene_perm=sd_, opts=o)
    ref = pd.run(torch.from_numpy(np.ascontiguousarray(W[:, inv])).cuda(), Pd, Cd, tol=0.0,
                 max_iter=3)
    torch.cuda.synchronize()
    want = ref.W[:, torch.from_numpy(s[0].astype(np.int64)).cuda()]
    err = (res.mean - want).abs().max().item()
    scale = max(1.0, want.abs().max().item())
    print(f"T={Ne} G={Na} 3 iterations: max|null instance - relabelled plain run| {err:.2e} "
          f"(max|W| {scale:.2f})")
    assert res.iters == [3] and ref.iters == 3
    assert err <= TOL * scale
    assert torch.count_nonzero(res.sd).item() == 0
