"""panda_pearson_noalloc, the entry point that allocates nothing (its scratch
is the library's per-GPU array), against panda_pearson with a workspace: two
calls in a row, the second on a smaller input, bit for bit; a size past the
scratch is refused before any device work."""
import ctypes as ct

import numpy as np
import pytest

from paper_1507_07039_amd import inputs as I

pytestmark = pytest.mark.gpu


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


def expression(torch, seed, G, S):
    E = I.random_dense(seed, (G, S), -2.0, 2.0)
    E[::97] = 0.75  # constant genes: correlation 0 with every other gene
    return torch.from_numpy(np.ascontiguousarray(E, dtype=np.float32)).cuda()


def test_noalloc_matches_workspace_entry_point(torch, pd, oracle):
    # the realistic expression size first, then a smaller ragged one: the
    # second call runs on scratch the first one left behind
    for G, S, seed in ((18000, 200, 7039), (333, 37, 11)):
        E = expression(torch, seed, G, S)
        want = pd.pearson(E)
        C = torch.full((G, G + 5), -7.0, dtype=torch.float32, device="cuda")
        got = pd.pearson_noalloc(E, C, ldc=G + 5)
        torch.cuda.synchronize()
        assert torch.equal(got[:, :G], want), (G, S)
        assert torch.all(got[:, G:] == -7.0)  # columns past G untouched
        print(f"G={G} S={S}: panda_pearson_noalloc equals panda_pearson bit for bit")
    # the smaller case against the FP64 oracle as well
    Eh = E.cpu().numpy().astype(np.float64)
    ref = oracle.pearson(Eh)
    assert np.abs(got[:, :G].cpu().numpy().astype(np.float64) - ref).max() <= 1e-5


def test_noalloc_refuses_sizes_past_its_scratch(torch, pd):
    lib = pd.load_library()
    G, S = 60000, 300
    assert lib.panda_pearson_workspace_bytes(G, S) > pd.NOALLOC_SCRATCH_BYTES
    dummy = torch.zeros(16, dtype=torch.float32, device="cuda")
    # rejected on the host from the sizes alone; the buffers are never touched
    st = lib.panda_pearson_noalloc(dummy.data_ptr(), G, S, S, dummy.data_ptr(), G,
                                   ct.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == pd.ERR_ARG
    assert b"scratch" in lib.panda_last_error()
    torch.cuda.synchronize()
    assert torch.all(dummy == 0)
