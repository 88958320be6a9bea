"""GPU test helpers: run tg_count through the C-ABI binding on numpy inputs."""
import sys

import numpy as np


def device():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(g_row_ptr, g_col_idx, g_types):
    import torch
    dev = device()
    return (torch.from_numpy(np.ascontiguousarray(g_row_ptr, dtype=np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(g_col_idx, dtype=np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(g_types, dtype=np.uint8)).to(dev))


def gpu_count(row_ptr, col_idx, types, L, per_edge=True, **kw):
    import torch

    import paper_1901_10026_amd as tg
    rp, ci, ty = to_dev(row_ptr, col_idx, types)
    g, rows, ends = tg.count(rp, ci, ty, L, per_edge=per_edge, **kw)
    torch.cuda.synchronize()
    g = g.cpu().numpy().view(np.uint64) if g is not None else None
    rows = rows.cpu().numpy().view(np.uint64) if rows is not None else None
    ends = ends.cpu().numpy() if ends is not None else None
    return g, rows, ends


def note(msg):
    """Progress line: printed, and appended to gpurun_out/gpu_tests.log under
    the repository root, so that a long GPU test is seen to progress even
    while pytest captures its output."""
    print(msg, flush=True)
    sys.stdout.flush()
    try:
        import os
        import time
        out = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
        os.makedirs(out, exist_ok=True)
        with open(os.path.join(out, "gpu_tests.log"), "a") as f:
            f.write(f"{time.strftime('%H:%M:%S')} {msg}\n")
    except OSError:
        pass
