"""The paper's run-time experiment (Table I) workload: random square W with
P = C = identity.  The GPU runs it as the message-passing procedure itself
(single networks and one batch of networks); parity against the FP64 oracle
at the smallest size of the table, and the timing driver end to end at a
reduced network count."""
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


N = 125
SEEDS = [1000 * N + k for k in range(3)]


def test_single_and_batched_match_oracle(torch, pd, oracle):
    """N = 125: each network to convergence on the GPU (panda_run, identity
    defaults) and in one batch, against the oracle from the same normalised
    FP32 inputs (max-abs W <= 1e-4, the same stopping iteration)."""
    eye = np.asarray(oracle.normalize(np.eye(N)), dtype=np.float32)
    Wd, refs = [], []
    for s in SEEDS:
        W0, _, _ = I.table1_priors(s, N)
        W = np.asarray(oracle.normalize(W0), dtype=np.float32)
        ref = oracle.run(W.astype(np.float64), eye.astype(np.float64), eye.astype(np.float64))
        Wd.append(torch.from_numpy(np.ascontiguousarray(W)).cuda())
        refs.append(ref)
    b = pd.Batch([(N, N)] * len(SEEDS))
    for i, W in enumerate(Wd):
        b.load(i, W)  # P, C: identity defaults, z-scored by the library
    b.run(graph=True)
    for i, (W, ref) in enumerate(zip(Wd, refs)):
        res = pd.run(W)
        torch.cuda.synchronize()
        err = np.abs(res.W.cpu().numpy().astype(np.float64) - ref.W).max()
        Wb, _, _, hb, tb = b.state(i)
        errb = np.abs(Wb.cpu().numpy().astype(np.float64) - ref.W).max()
        print(f"N={N} seed {SEEDS[i]}: iterations gpu {res.iters} batch {tb} oracle {ref.iters}; "
              f"max|W - oracle| single {err:.2e} batch {errb:.2e}")
        assert res.status == pd.OK and res.iters == ref.iters and tb == ref.iters
        assert err <= 1e-4 and errb <= 1e-4
    b.close()


def test_timing_driver(torch, pd):
    """The Table I driver end to end on two sizes with a few networks: every
    row carries times and iteration counts, and the batch converges in the
    same iterations as the single runs."""
    from paper_1507_07039_amd import table1
    rows = []
    for n in (125, 250):
        Ws = table1.networks(n, 3, torch, pd)
        secs, iters = table1.time_single(Ws, torch, pd)
        total, steps, biters = table1.time_batched(Ws, torch, pd)
        assert all(s > 0 for s in secs) and total > 0
        assert biters == iters and steps == max(iters)
        rows.append((n, iters))
    print("Table I driver:", rows)
