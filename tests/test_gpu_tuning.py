"""The batched driver's autotuner: tuned tile edge and persistent grid per size
bucket, kept across processes through a tuning file."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, empty, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sr():
    import torch

    import paper_2203_10879_amd as m

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def _batch(sr, sizes, seed0):
    mats = [synth.schur_test_matrix(n, seed=seed0 + i) for i, n in enumerate(sizes)]
    As = [dev(m["A"]) for m in mats]
    Qs = [dev(synth.lp_schur_start(m["A"])) for m in mats]
    Ts = [empty(n, n) for n in sizes]
    rc, infos = sr.schur_refine_batched(As, Qs, Ts)
    assert rc == 0, infos
    for m, qd, td in zip(mats, Qs, Ts):
        assert oracle.evaluate(m["A"], host(qd), host(td))["stril"] <= 1e-15


def test_tuning_table_save_load(sr, tmp_path):
    L = sr.lib()
    L.sr_tuning_reset()
    sizes = [20, 50, 100, 150, 200, 250]  # five size buckets
    runs0 = L.sr_tuning_runs()
    _batch(sr, sizes, 700)
    assert L.sr_tuning_runs() == runs0 + 5
    edges = [L.sr_batched_tile_edge(n) for n in sizes]
    grids = [L.sr_batched_tile_grid(n) for n in sizes]
    assert set(edges) <= {32, 64} and set(grids) <= {1, 2, 4, 8}, (edges, grids)
    path = str(tmp_path / "tuning.txt")
    assert L.sr_tuning_save(path.encode()) == 5
    lines = open(path).read().splitlines()
    assert lines[0].startswith("schur_refine batched tuning")
    rows = [ln.split() for ln in lines[1:]]
    assert len(rows) == 5 and all(len(r) == 5 for r in rows)
    assert sorted(int(r[1]) for r in rows) == [0, 1, 2, 3, 4]
    # a fresh table: nothing tuned; the file restores every choice without timing
    L.sr_tuning_reset()
    assert L.sr_batched_tile_edge(20) == -1
    assert L.sr_tuning_load(path.encode()) == 5
    assert [L.sr_batched_tile_edge(n) for n in sizes] == edges
    assert [L.sr_batched_tile_grid(n) for n in sizes] == grids
    runs1 = L.sr_tuning_runs()
    _batch(sr, sizes, 800)
    assert L.sr_tuning_runs() == runs1
    # lines of another device are kept on save and ignored on load
    with open(path, "a") as f:
        f.write("gfx000:other/1 0 32 8 1.0\n")
    assert L.sr_tuning_save(path.encode()) == 5
    assert any(ln.startswith("gfx000:other/1 ") for ln in open(path).read().splitlines())
    L.sr_tuning_reset()
    assert L.sr_tuning_load(path.encode()) == 5
    # a file without the header, or missing, is refused
    bad = str(tmp_path / "bad.txt")
    with open(bad, "w") as f:
        f.write("0 64 4 1.0\n")
    assert L.sr_tuning_load(bad.encode()) == -1
    assert L.sr_tuning_load(str(tmp_path / "none.txt").encode()) == -1
