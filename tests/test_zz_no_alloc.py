"""chap_best_shift_noalloc against chap_best_shift through the C ABI.

The no-allocation entry point carves every per-call buffer from one static
device array per GPU and launches the pass kernels without a graph. Its
results must equal chap_best_shift's bit for bit on consecutive calls whose
inputs shrink (the array keeps the previous call's contents), with and
without the cutoff row, on an all-integer staged instance with long columns
and on a small instance with continuous data; a problem that needs more
scratch than the array holds is rejected with CHAP_EINVAL.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import mipgen
import oracle

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def chap():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2605_05086_amd as c

    c.load_library()
    return c


def both(chap, G, mip, x, w, cutoff):
    import torch

    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()
    wd = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).cuda()
    a_x, a_s = G.best_shift(xd, wd, cutoff)
    b_x = torch.full_like(xd, np.nan)
    b_s = torch.full_like(xd, np.nan)
    G.best_shift_noalloc(xd, wd, b_x, b_s, cutoff)
    torch.cuda.synchronize()
    return a_x.cpu().numpy(), a_s.cpu().numpy(), b_x.cpu().numpy(), b_s.cpu().numpy()


def test_noalloc_equals_best_shift(chap):
    big = mipgen.powerlaw(91, n=200_000, m=100_000, nnz=2_000_000, cap=20_000)
    small = mipgen.random_mixed(92, n=500, m=300, max_row_nnz=8, integer_data=False, frac_bin=0.3, frac_int=0.3,
                                long_cols=3, long_deg=200)
    cases = [("2M-entry power-law", big, dict(chunk_min=1024)), ("continuous mixed", small, {})]
    for name, mip, opts in cases:
        G = chap.Problem(mip, **opts)
        P = oracle.OracleProblem(mip)
        for seed in (0, 1):
            x = mipgen.random_point(mip, seed)
            w = mipgen.random_weights(P.mp + 1, seed + 3, wmax=7)
            for cut in (math.inf, P.objective(x) - 2.5):
                say(f"noalloc {name} seed={seed} cutoff={cut}")
                ax, as_, bx, bs = both(chap, G, mip, x, w, cut)
                assert np.array_equal(as_, bs) and np.array_equal(ax, bx), name
                if seed == 0:
                    ox, os_ = P.best_shift(x, w, cut)
                    assert np.array_equal(bs, os_) and np.array_equal(bx, ox), name


def test_noalloc_rejects_large_problems(chap):
    import torch

    limit = chap.load_library().chap_best_shift_noalloc_max_bytes()
    assert limit == 64 << 20
    mip = mipgen.powerlaw(93, n=3_000_000, m=1_500_000, nnz=4_000_000, cap=20_000)  # 3 x 24 MB of columns alone
    G = chap.Problem(mip)
    x = torch.zeros(mip.n, dtype=torch.float64, device="cuda")
    w = torch.ones(G.mp + 1, dtype=torch.float32, device="cuda")
    out = torch.empty_like(x)
    say("noalloc rejects a problem beyond the scratch size")
    with pytest.raises(chap.ChapError, match="CHAP_EINVAL.*bytes of scratch"):
        G.best_shift_noalloc(x, w, out, out.clone())
