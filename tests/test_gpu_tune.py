"""The strip-height autotuner's cache on the GPU: a choice timed at setup is
saved with the device model in its key, and a loaded entry is used by a later
setup of that shape instead of timing the kernels again."""
import numpy as np
import pytest
import torch

from _helpers import make_case

pytestmark = pytest.mark.gpu


def test_tune_cache_entry_is_used(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_23804_amd as sgl
    print("[gpu-case] tuning cache", flush=True)
    _, kw = make_case(32, 3, 2, 0.25, 1e-2)
    sgl.tune_clear()
    h = sgl.Handle([sgl.ProblemData(**kw)], sgl.default_options(sweep_rows=0))
    tuned = [int(v) for v in h.sizes.sweep_rows[0]]
    assert all(v in (2, 4, 8) for v in tuned)
    assert sgl.tune_count() == 1
    saved = tmp_path / "tune.txt"
    sgl.tune_save(str(saved))
    lines = open(saved).read().splitlines()
    assert lines[0] == "sgkkt-tune 1" and len(lines) == 2
    f = lines[1].split()
    assert f[2:9] == ["32", "3", "2", "1", "0", "1", "0"] and [int(v) for v in f[9:]] == tuned
    # a different choice for the same key, loaded into an empty cache
    forced = [8 if v != 8 else 2 for v in tuned]
    edited = tmp_path / "edited.txt"
    with open(edited, "w") as out:
        out.write(lines[0] + "\n" + " ".join(f[:9] + [str(v) for v in forced]) + "\n")
    sgl.tune_clear()
    sgl.tune_load(str(edited))
    h2 = sgl.Handle([sgl.ProblemData(**kw)], sgl.default_options(sweep_rows=0))
    assert [int(v) for v in h2.sizes.sweep_rows[0]] == forced
    assert sgl.tune_count() == 1
    # the strip heights never change results: the operator agrees bit for bit
    x = torch.from_numpy(np.random.default_rng(1).uniform(-1, 1, size=h.kkt_elems)).to("cuda:0")
    y1, y2 = torch.zeros_like(x), torch.zeros_like(x)
    h.apply_kkt(x, y1)
    h2.apply_kkt(x, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    sgl.tune_clear()
