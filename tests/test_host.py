"""Host-only checks: the seeded generators follow their recipe, and the
benchmark refuses more than one GPU."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2101_05031_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [1, 2, 5, 25, 40, 52])
def test_kuhn_edge_count_and_uniqueness(n):
    e = synth.kuhn_edges(n)
    assert len(e) == synth.kuhn_edge_count(n)
    key = np.minimum(e[:, 0], e[:, 1]).astype(np.int64) * (n + 1) ** 3 + np.maximum(e[:, 0], e[:, 1])
    assert len(np.unique(key)) == len(e)


def test_kuhn_tets_are_covered():
    """Every tet of the Kuhn split (a path of +x, +y, +z steps through a cube)
    has its 6 edges in the edge set."""
    import itertools
    n = 2
    e = synth.kuhn_edges(n)
    s = {tuple(sorted(x)) for x in e.tolist()}
    idx = lambda i, j, k: (i * (n + 1) + j) * (n + 1) + k
    for perm in itertools.permutations(range(3)):
        v = [0, 0, 0]
        verts = [idx(*v)]
        for ax in perm:
            v[ax] += 1
            verts.append(idx(*v))
        for a, b in itertools.combinations(verts, 2):
            assert tuple(sorted((a, b))) in s


def test_bcc_counts():
    lat = synth.bcc_lattice(4, 5.0, 0.5)
    assert lat.n_nodes == 189 and lat.n_edges == 812
    L = np.linalg.norm(lat.nodes[lat.edges[:, 0]] - lat.nodes[lat.edges[:, 1]], axis=1)
    assert np.allclose(np.sort(np.unique(np.round(L, 9))), [5.0 * np.sqrt(3) / 2, 5.0])


def test_configs_are_seeded_and_shaped():
    lat, grid = synth.config("D4")
    lat2, _ = synth.config("D4")
    assert np.array_equal(lat.nodes, lat2.nodes) and np.array_equal(lat.weight, lat2.weight)
    assert lat.n_edges == 115075 and lat.nodes.dtype == np.float32
    assert grid.W == grid.H == 1024 and grid.n_slices == 64
    assert lat.R == pytest.approx(1.5)
    r = lat.radius
    assert r.min() >= 0.2 + 0.8 * 0.15 - 1e-6 and r.max() <= 1.0 + 1e-6
    # grid covers the bounding box grown by R with margin
    assert grid.x0 < lat.nodes[:, 0].min() - lat.R
    assert grid.x0 + grid.W * grid.dx > lat.nodes[:, 0].max() + lat.R


def test_blob_config_has_voids():
    lat, _ = synth.config("B3", scale=12)
    assert (lat.weight == 0).any() and (lat.weight > 0).any()
    assert lat.R == pytest.approx(0.9)


def test_weight_for_radius_rejects_out_of_range():
    with pytest.raises(ValueError):
        synth.weight_for_radius(1.5, 1.5)
    w = synth.weight_for_radius(np.array([0.2, 0.5, 0.9]), 1.5)
    assert np.all(np.diff(w) > 0)       # larger radius needs a larger weight


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
