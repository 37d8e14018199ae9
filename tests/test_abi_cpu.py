"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/sg.h, and rejects invalid problems on the host."""
import ctypes
import os
import re

import numpy as np
import pytest

import sg_inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "sg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char\*)\s+\*?\s*(sg_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    import paper_2512_23804_amd as sgl
    names = _declared_functions()
    assert len(names) >= 18
    raw = ctypes.CDLL(sgl._lib.LIB_PATH)
    for name in names:
        assert hasattr(raw, name), name
        assert name in sgl.SIGNATURES, name
    assert set(sgl.SIGNATURES) == set(names)


def test_default_options():
    import paper_2512_23804_amd as sgl
    o = sgl.default_options()
    assert o.rtol == 1e-8 and o.restart == 30 and o.cheb_steps == 5 and o.gmg_pre == 2 and o.gmg_post == 2
    assert o.precision == sgl.SG_PREC_FP64 and o.truncation_r == 0
    assert o.arnoldi == sgl.SG_ARNOLDI_DCGS2 and o.sweep_rows == 0 and o.use_graphs == 1
    assert o.mean_solver == sgl.SG_MEAN_MULTIGRID and o.richardson_steps == 1


def _pd(**kw):
    import paper_2512_23804_amd as sgl
    base = dict(n=16, M=4, P=3, sigma=0.2, beta=1e-2, y_target=sg_inputs.gaussian_bumps(16, 0))
    base.update(kw)
    return sgl.ProblemData(**base)


def test_validate_accepts_workload():
    import paper_2512_23804_amd as sgl
    assert sgl.validate(_pd()) == sgl.SG_OK
    assert sgl.validate(_pd(n=128, M=6, P=4, sigma=0.3, y_target=sg_inputs.gaussian_bumps(128, 1))) == sgl.SG_OK
    tgt = sg_inputs.moving_bump(64, 32, 1.0, 4)
    assert sgl.validate(_pd(n=64, n_t=32, beta=1e-3, y_target=tgt)) == sgl.SG_OK


@pytest.mark.parametrize("kw,code", [
    (dict(n=12), -1), (dict(n=4), -1), (dict(M=0), -1), (dict(M=17), -1), (dict(P=0), -1), (dict(P=9), -1),
    (dict(beta=0.0), -1), (dict(beta=-1.0), -1), (dict(gamma=-0.1), -1), (dict(beta=float("nan")), -3),
    (dict(sigma=0.9), -2),
])
def test_validate_rejects(kw, code):
    import paper_2512_23804_amd as sgl
    assert sgl.validate(_pd(**kw)) == code
    assert sgl.lib.sg_last_error().decode() != ""


def test_validate_nonfinite_target_and_custom_kappa():
    import paper_2512_23804_amd as sgl
    t = sg_inputs.gaussian_bumps(16, 0)
    t[7] = np.inf
    assert sgl.validate(_pd(y_target=t)) == sgl.SG_ERR_NONFINITE
    kap = np.zeros((5, 16, 16))
    kap[0] = 2.0
    kap[1] = 0.3
    assert sgl.validate(_pd(kappa=kap)) == sgl.SG_OK
    kap[1] = 1.2                      # 2 - sqrt(3) * 1.2 < 0: can vanish
    assert sgl.validate(_pd(kappa=kap)) == sgl.SG_ERR_NONCOERCIVE
    kap[1] = 0.3
    kap[0, 3, 3] = 2.5                # mean must be constant for the multigrid
    assert sgl.validate(_pd(kappa=kap)) == sgl.SG_ERR_INVALID


def test_validate_options():
    import paper_2512_23804_amd as sgl
    for kw in (dict(restart=0), dict(restart=40), dict(cheb_steps=-1), dict(cheb_steps=65), dict(truncation_r=6),
               dict(gmg_pre=0), dict(precision=3), dict(rtol=0.0), dict(sweep_rows=3), dict(sweep_rows=16),
               dict(arnoldi=2), dict(profile=9), dict(mean_solver=2), dict(richardson_steps=0),
               dict(richardson_steps=17)):
        assert sgl.validate(_pd(), sgl.default_options(**kw)) == sgl.SG_ERR_INVALID, kw
    # exact mass solves (cheb_steps = 0), exact mean-block solves and Richardson steps are valid
    for kw in (dict(cheb_steps=0), dict(mean_solver=sgl.SG_MEAN_EXACT), dict(richardson_steps=4)):
        assert sgl.validate(_pd(), sgl.default_options(**kw)) == sgl.SG_OK, kw


def test_setup_rejects_before_touching_the_device():
    import ctypes as C

    import paper_2512_23804_amd as sgl
    p = _pd(sigma=0.95)
    h = C.c_void_p()
    rc = sgl.lib.sg_setup(C.byref(p.c), 1, None, None, C.byref(h))
    assert rc == sgl.SG_ERR_NONCOERCIVE and not h.value
    rc = sgl.lib.sg_setup(C.byref(p.c), 0, None, None, C.byref(h))
    assert rc == sgl.SG_ERR_INVALID


def test_serving_stream_shapes_do_not_depend_on_the_rate():
    """The serving protocol replays one request mix at several arrival rates
    (all at once for capacity, then Poisson streams): the drawn shapes, fields
    and targets must be the same whatever the rate, and an infinite rate puts
    every arrival at time zero."""
    grids = (32, 64, 128, 256)
    mixes = [sg_inputs.serving_stream(64, seed=7, rate_per_s=r, grid_choices=grids)
             for r in (float("inf"), 4.5, 13.4)]
    keys = ("n", "M", "P", "sigma", "beta", "seed")
    for mix in mixes[1:]:
        assert [tuple(q[k] for k in keys) for q in mix] == [tuple(q[k] for k in keys) for q in mixes[0]]
    assert all(q["arrival"] == 0.0 for q in mixes[0])
    for mix in mixes[1:]:
        arr = np.array([q["arrival"] for q in mix])
        assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0.0)
    # the protocol's ranges
    q = mixes[0]
    assert {r["n"] for r in q} <= set(grids)
    assert all(4 <= r["M"] <= 8 and 2 <= r["P"] <= 4 and 0.1 <= r["sigma"] <= 0.3 for r in q)
    assert all(1e-6 <= r["beta"] <= 1e-1 for r in q)
    assert [r["seed"] for r in q] == list(range(1000, 1064))


def test_validate_lognormal_field():
    import paper_2512_23804_amd as sgl
    ln = dict(field=sgl.SG_FIELD_LOGNORMAL, y_target=sg_inputs.indicator_target(16))
    assert sgl.validate(_pd(**ln)) == sgl.SG_OK
    assert sgl.validate(_pd(field=2)) == sgl.SG_ERR_INVALID
    assert sgl.validate(_pd(corr_len=0.0, **ln)) == sgl.SG_ERR_INVALID
    kap = np.ones((5, 16, 16))
    assert sgl.validate(_pd(kappa=kap, **ln)) == sgl.SG_ERR_INVALID
    # a log-normal field may use sigma large enough to break the affine field's coercivity
    assert sgl.validate(_pd(sigma=2.0, **ln)) == sgl.SG_OK
    # truncation up to n_A = C(M + 2P, 2P) terms (M = 4, P = 3: 210), the affine field up to M + 1
    assert sgl.validate(_pd(**ln), sgl.default_options(truncation_r=210)) == sgl.SG_OK
    assert sgl.validate(_pd(**ln), sgl.default_options(truncation_r=211)) == sgl.SG_ERR_INVALID
    assert sgl.validate(_pd(), sgl.default_options(truncation_r=6)) == sgl.SG_ERR_INVALID


def test_validate_hgsoc_option():
    import paper_2512_23804_amd as sgl
    o = sgl.default_options
    assert sgl.validate(_pd(), o(precond=sgl.SG_PRECOND_HGSOC)) == sgl.SG_OK
    assert sgl.validate(_pd(), o(precond=2)) == sgl.SG_ERR_INVALID
    # with the fused Chebyshev mass solves only; time-dependent problems take
    # it per time step (Algorithm 4)
    assert sgl.validate(_pd(), o(precond=sgl.SG_PRECOND_HGSOC, cheb_steps=12)) == sgl.SG_ERR_INVALID
    assert sgl.validate(_pd(), o(precond=sgl.SG_PRECOND_HGSOC, cheb_steps=0)) == sgl.SG_ERR_INVALID
    tgt = np.stack([sg_inputs.gaussian_bumps(16, 0)] * 3)
    assert sgl.validate(_pd(n_t=3, y_target=tgt), o(precond=sgl.SG_PRECOND_HGSOC)) == sgl.SG_OK


TUNE_LINES = ["gfx950:sramecc+:xnack- 256 128 6 4 1 0 1 0 4 4 8",
              "gfx950:sramecc+:xnack- 256 512 8 3 1 0 2 1 2 4 4"]


def _tune_file(path, lines, magic="sgkkt-tune 1"):
    with open(path, "w") as f:
        f.write(magic + "\n" + "\n".join(lines) + "\n")


def test_tune_cache_round_trip(tmp_path):
    """The strip-height cache file: a load merges its entries, a save writes
    them back in the same format, a clear empties the cache (no device)."""
    import paper_2512_23804_amd as sgl
    sgl.tune_clear()
    assert sgl.tune_count() == 0
    src = tmp_path / "in.txt"
    _tune_file(src, TUNE_LINES)
    sgl.tune_load(str(src))
    assert sgl.tune_count() == 2
    out = tmp_path / "out.txt"
    sgl.tune_save(str(out))
    lines = open(out).read().splitlines()
    assert lines[0] == "sgkkt-tune 1" and sorted(lines[1:]) == sorted(TUNE_LINES)
    # an entry with the same key replaces the cached one
    _tune_file(src, [TUNE_LINES[0].rsplit(" ", 3)[0] + " 2 2 2"])
    sgl.tune_load(str(src))
    assert sgl.tune_count() == 2
    sgl.tune_save(str(out))
    assert TUNE_LINES[0].rsplit(" ", 3)[0] + " 2 2 2" in open(out).read().splitlines()
    sgl.tune_clear()
    assert sgl.tune_count() == 0


@pytest.mark.parametrize("lines,magic", [
    (["gfx950 256 128 6 4 1 0 1 0 4 4 3"], "sgkkt-tune 1"),        # strip height not in {2, 4, 8}
    (["gfx950 256 128 6 4 1 0 1 0 4 4"], "sgkkt-tune 1"),          # missing field
    (["gfx950 256 128 6 4 1 0 1 0 4 4 8 1"], "sgkkt-tune 1"),      # extra field
    (["gfx950 256 128 6 4 1 0 3 0 4 4 8"], "sgkkt-tune 1"),        # batch class 3
    (TUNE_LINES, "sgkkt-tune 2"),                                   # wrong version line
])
def test_tune_cache_rejects_malformed_files(tmp_path, lines, magic):
    import paper_2512_23804_amd as sgl
    sgl.tune_clear()
    _tune_file(tmp_path / "bad.txt", [TUNE_LINES[1]] + lines, magic)
    with pytest.raises(sgl.SGError) as e:
        sgl.tune_load(str(tmp_path / "bad.txt"))
    assert e.value.code == sgl.SG_ERR_INVALID
    assert sgl.tune_count() == 0          # nothing merged from a file that does not parse
    with pytest.raises(sgl.SGError):
        sgl.tune_load(str(tmp_path / "missing.txt"))
    with pytest.raises(sgl.SGError):
        sgl.tune_save(str(tmp_path / "no_such_dir" / "x.txt"))


def test_tune_cache_environment_file(tmp_path):
    """SG_TUNE_CACHE: a fresh process merges the file it names at its first
    use of the cache (here a count, which touches no device)."""
    import subprocess
    import sys
    src = tmp_path / "cache.txt"
    _tune_file(src, TUNE_LINES)
    env = dict(os.environ, SG_TUNE_CACHE=str(src))
    code = ("import paper_2512_23804_amd as s; print(s.tune_count())")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "2"
