"""The autotuners only change launch shapes: counts stay identical."""
import json

import numpy as np
import pytest

import graphgen
from _gpu import to_dev

pytestmark = pytest.mark.gpu


def test_autotune_count_keeps_counts(tmp_path):
    import torch

    import paper_1901_10026_amd as tg
    g = graphgen.chung_lu_small()
    rp, ci, ty = to_dev(g.row_ptr, g.col_idx, g.types)
    g0, r0, _ = tg.count(rp, ci, ty, g.L)
    out_g = torch.empty_like(g0)
    out_e = torch.empty_like(r0)
    t, ms = tg.autotune(rp, ci, ty, g.L, out_g, out_e, schedule="degree")
    assert ms > 0
    g1, r1, _ = tg.count(rp, ci, ty, g.L, tuning=t)
    torch.cuda.synchronize()
    assert torch.equal(g0.view(torch.int64), g1.view(torch.int64))
    assert torch.equal(r0.view(torch.int64), r1.view(torch.int64))
    path = tmp_path / "tuning.json"
    key = tg.tuning_cache_key("count", workload="cl-2k", schedule="degree")
    tg.save_tuning(path, key, t)
    assert tg.load_tuning(path, key).as_dict() == t.as_dict()
    assert key in json.load(open(path))


def test_autotune_batch_keeps_counts():
    import torch

    import paper_1901_10026_amd as tg
    b = graphgen.batch_gnp(400, 5, 500, 0.02, 0.3, 2, 8, 77)
    dev = torch.device("cuda:0")
    key_off = tg.key_offsets(b.L)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)
    args = (t(b.node_off, np.int64), t(b.slot_off, np.int64), t(b.row_ptr, np.int32), t(b.col_idx, np.int32),
            t(b.types, np.uint8), t(b.L, np.uint8), t(key_off, np.int64))
    base = tg.count_batch(*args).clone()
    out = torch.empty_like(base)
    tuning, ms = tg.autotune_batch(*args, out)
    assert ms > 0
    wmax = {0: 1, 1: 2, 2: 2, 3: 4, 4: 4, 5: 8}
    for w in range(1, 9):
        assert wmax[tuning.batch_variant[w]] >= w
    again = tg.count_batch(*args, tuning=tuning)
    torch.cuda.synchronize()
    assert torch.equal(again.view(torch.int64), base.view(torch.int64))
