"""Via minimisation on the GPU: a 40 x 40 routing instance annealed as a
weighted max-cut, bit-exact to the oracle, with via counts from the direct
definition (a on cut edges, b on uncut ones)."""
import numpy as np
import pytest

import oracle as O
from paper_1807_10750_amd import graphs as G
from paper_1807_10750_amd import via

pytestmark = pytest.mark.gpu


def test_via_instance_anneal(I=None):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_10750_amd import ising as I
    n, u, v, a, b = G.via_instance(40, 40, 3, 7)
    g, B = via.via_graph(n, u, v, a, b)
    R, M, seed = 8, 300, 13
    gr = I.Graph.from_csr(g, replicas=R)
    gr.randomize(seed)
    gr.anneal(I.make_schedule(0.2, 0.0, M), seed, I.MODE_DETERMINISTIC)
    s = gr.spins()
    c, _ = gr.cut()
    gr.close()
    so, Co, _ = O.solve(g, seed, 0.2, 0.0, M, R=R)
    assert np.array_equal(s, so) and np.array_equal(c, Co)
    direct = np.array([int(np.where(s[r, u] != s[r, v], a, b).sum()) for r in range(R)])
    assert np.array_equal(via.vias_from_cut(B, c), direct)
    # far fewer vias than a random layer assignment
    rnd = G.random_spins(n, 64, 1)
    rnd_vias = np.array([int(np.where(x[u] != x[v], a, b).sum()) for x in rnd])
    assert direct.max() < rnd_vias.min()
