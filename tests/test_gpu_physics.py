"""Physics and state-handling checks of the device sweeps.

* Magnetization vs temperature (Algorithm 1's observable; the paper's
  validation plots |m|(T) for several L): on a 4^3 lattice with M = 256 and
  mu = 0 the double-exchange ferromagnet must be ordered at T = 0.02t and
  disordered at T = 1t, with |m| non-increasing in between (within noise).
* Checkpoint / resume: angles + proposal counter are the whole chain state, so
  1 sweep + save/restore + 1 sweep equals 2 sweeps bit for bit.
* Determinism: the same seeded run twice gives identical results.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1303_6016_amd as g
    g.lib()
    return g


def test_magnetization_falls_with_temperature(g):
    temps = [0.02, 0.05, 0.1, 0.2, 0.4, 1.0]
    chains = []
    for i, T in enumerate(temps):
        ch = g.Chain(g.Params(L=4, M=256, beta=1.0 / T, seed=31, chain_id=i))
        ch.init_spins(g.INIT_FM)
        chains.append(ch)
    b = g.Batch(chains)
    b.sweep(20)                       # warm-up sweeps, discarded
    mag, acc = b.sweep(60)
    b.close()
    m = mag.mean(axis=1)
    print("T:", temps, "\n<|m|>:", np.round(m, 3), "\nacceptance:",
          np.round(acc / (60 * 64), 3), flush=True)
    assert m[0] > 0.85
    assert m[-1] < 0.35
    assert np.all(np.diff(m) < 0.05)
    assert acc[0] < acc[-1]           # proposals are accepted more often when hot


def test_checkpoint_resume_is_bit_exact(g):
    def make():
        ch = g.Chain(g.Params(L=4, M=128, beta=8.0, seed=5, chain_id=2))
        ch.init_spins(g.INIT_RANDOM)
        return ch
    a = make()
    ma, _ = a.sweep(2)
    b = make()
    mb1, _ = b.sweep(1)
    th, ph = b.get_spins()
    idx = b.get_counter()
    c = make()                        # a fresh chain restored from the checkpoint
    c.set_spins(th, ph)
    c.set_counter(idx)
    mc, _ = c.sweep(1)
    assert idx == 64
    assert np.array_equal(a.get_spins()[0], c.get_spins()[0])
    assert np.array_equal(a.get_spins()[1], c.get_spins()[1])
    assert ma[1] == mc[0] and ma[0] == mb1[0]


def test_runs_are_deterministic(g):
    out = []
    for _ in range(2):
        ch = g.Chain(g.Params(L=6, M=128, beta=10.0, precision=1, seed=8))
        ch.init_spins(g.INIT_RANDOM)
        recs = [ch.step() for _ in range(10)]
        out.append([(r.site, r.dseff, r.accepted) for r in recs])
    assert out[0] == out[1]
