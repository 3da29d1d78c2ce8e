"""The GPU parameter search (paper_math_9907190_amd/tune.py): its factor
equals the oracle's for the same parameters and start (the cycles agree to
1e-12, so the residual-norm ratios do too), and the search from the same
point ends at the oracle search's parameters."""
import numpy as np
import pytest
import torch

from paper_math_9907190_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_math_9907190_amd import dmg as D, tune
    return D, tune


def oracle_factor(orc, tune, dim, n, p, cycles=30, tail=10, seed=0):
    u = W.uniform(dim, n, seed)
    f = np.zeros_like(u)
    norms = []
    for k in range(cycles + 1):
        norms.append(orc.relres(u, f))
        if k < cycles:
            u = orc.vcycle(u, f, p)
    return tune.tail_factor(norms, tail)


@pytest.mark.parametrize("dim,n,p", [(2, 64, (1.0,)), (2, 64, (1.052,)), (2, 512, (1.1,)),
                                     (3, 16, (1.11, 1.42, 1.08, 0.99)), (3, 64, (1.0, 1.0, 1.0, 1.0))])
def test_factor_matches_oracle(mods, orc, dim, n, p):
    D, tune = mods
    print("factor dim=%d n=%d p=%s" % (dim, n, p), flush=True)
    g = tune.gpu_factor(dim, n, p)
    o = oracle_factor(orc, tune, dim, n, p)
    assert abs(g - o) <= 1e-9 * o, (g, o)


def test_search_matches_oracle_search(mods, orc):
    D, tune = mods
    print("search 65^2", flush=True)
    pg, fg, ng = tune.tune_p(2, 64, p0=(1.0,))
    po, fo, no = tune.nelder_mead(lambda p: oracle_factor(orc, tune, 2, 64, p) if min(p) > 0 else 1e3, (1.0,))
    assert abs(pg[0] - po[0]) < 1e-3 and abs(fg - fo) < 1e-6, (pg, po, fg, fo)
