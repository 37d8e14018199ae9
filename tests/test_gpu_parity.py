"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (element-wise, scaled by the reference's max-norm):
  * multi-index set and triple-product sparsity: bit-exact;
  * FP64 operator / KKT / preconditioner applies: 1e-12;
  * solutions: each block within 1e-8 of the direct solve (solved to 1e-12);
  * FP32 applies: 1e-5 (single-precision rounding of O(10)-term sums).
"""
import sys

import numpy as np
import pytest

from oracle import basis, fem, kkt, precond

from _helpers import canonical_to_kkt, kkt_to_canonical, make_case, rel_max, ring_is_zero

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    import paper_2512_23804_amd as sgl
    return sgl


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _setup(lib_kw_list, **opt):
    sgl = _lib()
    probs = [sgl.ProblemData(**kw) for kw in lib_kw_list]
    return sgl.Handle(probs, sgl.default_options(**opt))


SHAPES = [
    # n, M, P, sigma, beta, gamma, n_t
    (8, 1, 1, 0.3, 1e-2, 0.0, 1),
    (16, 4, 3, 0.2, 1e-2, 0.0, 1),       # the small steady workload
    (32, 3, 2, 0.25, 1e-4, 0.5, 1),
    (16, 2, 3, 0.3, 1e-3, 0.0, 4),
    (8, 3, 2, 0.2, 1e-2, 0.7, 3),
]


@pytest.mark.parametrize("shape", SHAPES)
def test_multiindex_and_gtable(shape):
    n, M, P, sigma, beta, gamma, nt = shape
    _dev()
    _say(f"tables {shape}")
    prob, kw = make_case(n, M, P, sigma, beta, gamma, nt)
    h = _setup([kw])
    A = basis.multi_indices(M, P)
    assert np.array_equal(h.multiindex(), A)
    idx, val = h.gtable()
    G = basis.triple_product_matrices(M, P)
    # rebuild dense G_k from the library's table and compare pattern and values
    for k in range(1, M + 1):
        Gl = np.zeros_like(G[k])
        for j in range(A.shape[0]):
            for s in range(2):
                i = idx[j, k - 1, s]
                if i >= 0:
                    Gl[i, j] = val[j, k - 1, s]
        assert np.array_equal(Gl != 0, G[k] != 0)
        assert np.max(np.abs(Gl - G[k])) < 1e-14
    assert h.level_offsets == list(basis.level_offsets(M, P))


@pytest.mark.parametrize("shape", SHAPES)
def test_operator_apply(shape):
    n, M, P, sigma, beta, gamma, nt = shape
    dev = _dev()
    _say(f"operator apply {shape}")
    prob, kw = make_case(n, M, P, sigma, beta, gamma, nt)
    sg = kkt.setup(prob)
    h = _setup([kw])
    rng = np.random.default_rng(1)
    nvec = 2
    X = rng.uniform(-1, 1, size=(nvec, max(nt, 1), sg.n_xi, (n + 1) ** 2))
    Xd = torch.from_numpy(X).to(dev)
    Yd = torch.full_like(Xd, np.nan)
    h.apply_operator(Xd, Yd)
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy()
    assert ring_is_zero(Y, n)
    for v in range(nvec):
        for t in range(max(nt, 1)):
            ref = kkt.operator_apply(sg, fem.extract(X[v, t], n))
            assert rel_max(fem.extract(Y[v, t], n), ref) < 1e-12
    # FP32 path
    Yf = torch.zeros_like(Xd, dtype=torch.float32)
    h.apply_operator(Xd.float(), Yf)
    torch.cuda.synchronize()
    ref = kkt.operator_apply(sg, fem.extract(X[0, 0].astype(np.float32).astype(np.float64), n))
    assert rel_max(fem.extract(Yf.cpu().numpy()[0, 0].astype(np.float64), n), ref) < 1e-5


@pytest.mark.parametrize("shape", SHAPES)
def test_kkt_apply(shape):
    n, M, P, sigma, beta, gamma, nt = shape
    dev = _dev()
    _say(f"kkt apply {shape}")
    prob, kw = make_case(n, M, P, sigma, beta, gamma, nt, y0=nt > 1)
    sg = kkt.setup(prob)
    h = _setup([kw])
    K = kkt.kkt_matrix(sg)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, size=K.shape[0])
    xd = torch.from_numpy(kkt_to_canonical(sg, x)).to(dev)
    yd = torch.zeros_like(xd)
    h.apply_kkt(xd, yd)
    torch.cuda.synchronize()
    y = canonical_to_kkt(sg, yd.cpu().numpy())
    assert rel_max(y, K @ x) < 1e-12
    # right-hand side
    bd = torch.zeros_like(xd)
    h.rhs(bd)
    assert rel_max(canonical_to_kkt(sg, bd.cpu().numpy()), kkt.rhs(sg)) < 1e-14


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("r_trunc", [1, 0])
def test_precond_apply(shape, r_trunc):
    n, M, P, sigma, beta, gamma, nt = shape
    dev = _dev()
    _say(f"precond {shape} r={r_trunc}")
    prob, kw = make_case(n, M, P, sigma, beta, gamma, nt)
    sg = kkt.setup(prob)
    h = _setup([kw], truncation_r=r_trunc)
    rng = np.random.default_rng(3)
    m = kkt.kkt_matrix(sg).shape[0]
    r = rng.uniform(-1, 1, size=m)
    rd = torch.from_numpy(kkt_to_canonical(sg, r)).to(dev)
    zd = torch.full_like(rd, np.nan)
    h.precond_apply(rd, zd)
    torch.cuda.synchronize()
    z = canonical_to_kkt(sg, zd.cpu().numpy())
    ref = precond.precond_apply(sg, r, precond.make_inner(sg), r_trunc if r_trunc else M + 1)
    for a, b in zip(kkt.split(sg, z), kkt.split(sg, ref)):
        assert rel_max(a, b) < 1e-12
    assert ring_is_zero(zd.cpu().numpy(), n)


def test_precond_multi_rhs_shares_one_member():
    dev = _dev()
    _say("precond multi-rhs")
    prob, kw = make_case(16, 3, 2, 0.3, 1e-2)
    sg = kkt.setup(prob)
    h = _setup([kw])
    rng = np.random.default_rng(4)
    m = kkt.kkt_matrix(sg).shape[0]
    rs = [rng.uniform(-1, 1, size=m) for _ in range(3)]
    rd = torch.from_numpy(np.concatenate([kkt_to_canonical(sg, r) for r in rs])).to(dev)
    zd = torch.zeros_like(rd)
    h.precond_apply(rd, zd)
    torch.cuda.synchronize()
    Z = zd.cpu().numpy().reshape(3, -1)
    inner = precond.make_inner(sg)
    for i in range(3):
        assert rel_max(canonical_to_kkt(sg, Z[i]), precond.precond_apply(sg, rs[i], inner)) < 1e-12


@pytest.mark.parametrize("arnoldi", [0, 1])
@pytest.mark.parametrize("shape", [SHAPES[1], SHAPES[2], SHAPES[3]])
def test_solve_matches_direct(shape, arnoldi):
    """FGMRES with either orthogonalisation (0: delayed reorthogonalisation,
    1: Gram-Schmidt twice) reaches the oracle's direct solution."""
    n, M, P, sigma, beta, gamma, nt = shape
    dev = _dev()
    _say(f"solve {shape} arnoldi={arnoldi}")
    prob, kw = make_case(n, M, P, sigma, beta, gamma, nt, y0=nt > 1)
    sg = kkt.setup(prob)
    h = _setup([kw], rtol=1e-12, max_iter=400, arnoldi=arnoldi)
    xd = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
    rc, info = h.solve(xd)
    torch.cuda.synchronize()
    assert rc == 0 and info[0].converged == 1 and info[0].rel_res_true <= 1e-12
    x = canonical_to_kkt(sg, xd.cpu().numpy())
    ref = kkt.solve_direct(sg)
    for a, b in zip(kkt.split(sg, x), kkt.split(sg, ref)):
        assert rel_max(a, b) < 1e-8
    # the oracle's own residual of the GPU solution
    K = kkt.kkt_matrix(sg)
    b = kkt.rhs(sg)
    assert np.linalg.norm(b - K @ x) / np.linalg.norm(b) < 1e-11


@pytest.mark.parametrize("shape", [(16, 3, 2, 0.0, 1e-2, 0.0, 1), (16, 2, 2, 0.0, 1e-3, 0.0, 3)])
def test_deterministic_field_stays_in_the_mean(shape):
    """sigma = 0: every fluctuation mode of the field vanishes, so neither the
    KKT operator nor the preconditioner couples chaos columns, and the
    right-hand side lives in column 0.  The solution is exactly zero in every
    other column (steady and time-dependent) and column 0 is the oracle's
    direct solution of the deterministic problem."""
    n, M, P, sigma, beta, gamma, nt = shape
    dev = _dev()
    _say(f"deterministic field {shape}")
    prob, kw = make_case(n, M, P, sigma, beta, gamma, nt, y0=nt > 1)
    sg = kkt.setup(prob)
    h = _setup([kw], rtol=1e-12, max_iter=400)
    xd = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
    rc, info = h.solve(xd)
    torch.cuda.synchronize()
    assert rc == 0 and info[0].converged == 1 and info[0].rel_res_true <= 1e-12
    x = canonical_to_kkt(sg, xd.cpu().numpy())
    ref = kkt.solve_direct(sg)
    for a, b in zip(kkt.split(sg, x), kkt.split(sg, ref)):
        higher = a[1:] if nt == 1 else a[:, 1:]
        assert np.all(higher == 0.0)
        mean, mean_ref = (a[0], b[0]) if nt == 1 else (a[:, 0], b[:, 0])
        assert rel_max(mean, mean_ref) < 1e-8


@pytest.mark.parametrize("basis_fp32", [1, 0])
def test_solve_fp32_refine_reaches_fp64_accuracy(basis_fp32):
    """FP64 refinement around FP32-storage inner cycles (the basis in FP32 or
    FP64 storage) reaches the direct solution to FP64 accuracy."""
    dev = _dev()
    _say(f"solve fp32 refine, basis_fp32={basis_fp32}")
    prob, kw = make_case(16, 4, 3, 0.2, 1e-2)
    sg = kkt.setup(prob)
    h = _setup([kw], rtol=1e-12, max_iter=600, precision=1, basis_fp32=basis_fp32)
    xd = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
    rc, info = h.solve(xd)
    assert rc == 0 and info[0].rel_res_true <= 1e-12 and info[0].outer_refinements >= 1
    x = canonical_to_kkt(sg, xd.cpu().numpy())
    ref = kkt.solve_direct(sg)
    for a, b in zip(kkt.split(sg, x), kkt.split(sg, ref)):
        assert rel_max(a, b) < 1e-8


@pytest.mark.parametrize("shape", [SHAPES[1], SHAPES[2], SHAPES[3], (64, 6, 2, 0.2, 1e-2, 0.0, 1)])
def test_sweep_rows_bit_identical(shape):
    """The strip heights the autotuner chooses between (2, 4, 8 node rows) give
    bit-identical operator, KKT and preconditioner applies, FP64 and FP32, and
    identical solves; the autotuned handle reports a valid choice."""
    n, M, P, sigma, beta, gamma, nt = shape
    dev = _dev()
    _say(f"sweep rows {shape}")
    prob, kw = make_case(n, M, P, sigma, beta, gamma, nt, y0=nt > 1)
    rng = np.random.default_rng(11)
    outs = {}
    for rows in (2, 4, 8, 0):
        h = _setup([kw], rtol=1e-10, sweep_rows=rows, precision=2)
        tuned = [list(r) for r in h.sizes.sweep_rows]
        assert all(v in (2, 4, 8) for r in tuned for v in r), tuned
        if rows:
            assert all(v == rows for r in tuned for v in r), tuned
        x = torch.from_numpy(rng.uniform(-1, 1, size=h.kkt_elems)) if not outs else outs["x"]
        outs["x"] = x
        xd = x.to(dev)
        res = []
        for dt in (torch.float64, torch.float32):
            xi = xd.to(dt)
            for fn in (h.apply_kkt, h.precond_apply):
                y = torch.zeros_like(xi)
                fn(xi, y)
                res.append(y)
            xo = xi[: h.sizes.block_elems].contiguous()
            yo = torch.zeros_like(xo)
            h.apply_operator(xo, yo)
            res.append(yo)
        sol = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
        rc, info = h.solve(sol)
        assert rc == 0
        res.append(sol)
        torch.cuda.synchronize()
        if "ref" not in outs:
            outs["ref"] = res
        else:
            for a, b in zip(res, outs["ref"]):
                assert torch.equal(a, b), rows
        h.close()


def test_solve_fp32_preconditioner_tracks_fp64():
    """FP32 preconditioner inside FP64 FGMRES: reaches the direct solution and
    needs about the FP64 iteration count (the operator stays FP64)."""
    dev = _dev()
    _say("solve fp32 preconditioner")
    prob, kw = make_case(32, 4, 3, 0.3, 1e-4, seed=3)
    sg = kkt.setup(prob)
    its = {}
    for prec in (0, 2):
        h = _setup([kw], rtol=1e-12, max_iter=600, precision=prec)
        xd = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
        rc, info = h.solve(xd)
        assert rc == 0 and info[0].rel_res_true <= 1e-12
        its[prec] = info[0].iters
        if prec == 2:
            x = canonical_to_kkt(sg, xd.cpu().numpy())
            ref = kkt.solve_direct(sg)
            for a, b in zip(kkt.split(sg, x), kkt.split(sg, ref)):
                assert rel_max(a, b) < 1e-8
    assert its[2] <= its[0] + 2 + its[0] // 10, its


def test_batch_results_equal_alone():
    """Members of one batch (different sigma, beta, targets) give bit-identical
    results to solving each alone."""
    dev = _dev()
    _say("batch invariance")
    params = [(0.2, 1e-2, 0), (0.3, 1e-4, 1), (0.1, 1e-3, 2)]
    kws = [make_case(16, 3, 2, s, b, seed=sd)[1] for s, b, sd in params]
    for prec in (0, 1, 2):
        hb = _setup(kws, rtol=1e-8, precision=prec)
        xb = torch.zeros(3 * hb.kkt_elems, dtype=torch.float64, device=dev)
        rc, infos = hb.solve(xb)
        assert rc == 0
        for i, kw in enumerate(kws):
            ha = _setup([kw], rtol=1e-8, precision=prec)
            xa = torch.zeros(ha.kkt_elems, dtype=torch.float64, device=dev)
            rca, infa = ha.solve(xa)
            assert rca == 0 and infa[0].iters == infos[i].iters
            assert torch.equal(xa, xb[i * ha.kkt_elems:(i + 1) * ha.kkt_elems])
            # the bytes model is per member: the same alone and in the batch, and at
            # least an operator apply and a preconditioner of KKT-apply size per iteration
            assert infa[0].bytes_moved == infos[i].bytes_moved
            assert infos[i].bytes_moved > infos[i].iters * 2 * 6 * 4 * hb.block_elems


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_members_stop_on_the_device(precision):
    """A batch whose members need very different iteration counts (several
    restart cycles for one, one cycle for another), on a created stream with
    per-iteration graphs: the device clears each member's flag when its
    estimate converges and later launches skip it; every member still gives
    the iterations and the bit-identical result of its alone solve."""
    dev = _dev()
    _say(f"device-side stop precision={precision}")
    sgl = _lib()
    params = [(0.1, 1e-1, 3), (0.3, 1e-6, 4), (0.2, 1e-3, 5)]
    kws = [make_case(16, 3, 2, s, b, seed=sd)[1] for s, b, sd in params]
    stream = torch.cuda.Stream()
    opts = dict(rtol=1e-10, precision=precision, use_graphs=1, max_iter=400)
    hb = sgl.Handle([sgl.ProblemData(**kw) for kw in kws], sgl.default_options(**opts), stream=stream)
    xb = torch.zeros(3 * hb.kkt_elems, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()              # the solve writes xb on `stream`
    for _ in range(2):                    # the second solve replays the captured graphs
        rc, infos = hb.solve(xb)
        assert rc == 0
    its = [inf.iters for inf in infos]
    assert max(its) > 30 and min(its) < max(its), its
    for i, kw in enumerate(kws):
        ha = sgl.Handle([sgl.ProblemData(**kw)], sgl.default_options(**opts), stream=stream)
        xa = torch.zeros(ha.kkt_elems, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        rca, infa = ha.solve(xa)
        assert rca == 0 and infa[0].iters == infos[i].iters
        assert torch.equal(xa, xb[i * ha.kkt_elems:(i + 1) * ha.kkt_elems])


def test_delayed_reorthogonalisation_tracks_cgs2():
    """Across restarts and a hard beta, the delayed-reorthogonalisation Arnoldi
    needs about the iterations of Gram-Schmidt twice and reaches the same
    true residual; a short restart exercises the end-of-cycle commit."""
    dev = _dev()
    _say("dcgs2 vs cgs2")
    prob, kw = make_case(32, 4, 3, 0.3, 1e-6, seed=5)
    for restart in (30, 7):
        its = []
        for arnoldi in (0, 1):
            h = _setup([kw], rtol=1e-10, restart=restart, max_iter=600, arnoldi=arnoldi)
            x = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
            rc, info = h.solve(x)
            assert rc == 0 and info[0].converged == 1 and info[0].rel_res_true <= 1e-10
            its.append(info[0].iters)
        assert abs(its[0] - its[1]) <= 2 + its[1] // 10, its


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_graph_replay_matches_direct_launches(precision):
    """Solves on a created stream replay cached per-iteration graphs after the
    first cycle; three consecutive solves with graphs and one without must be
    bit-identical."""
    dev = _dev()
    _say(f"graph replay precision={precision}")
    sgl = _lib()
    prob, kw = make_case(16, 3, 2, 0.3, 1e-3)
    stream = torch.cuda.Stream()
    outs = []
    for use_graphs in (1, 1, 1, 0):
        if not outs or use_graphs == 0:
            h = sgl.Handle([sgl.ProblemData(**kw)], sgl.default_options(rtol=1e-10, precision=precision,
                                                                        use_graphs=use_graphs), stream=stream)
        x = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()          # x is read and written on `stream`
        rc, info = h.solve(x)
        assert rc == 0 and info[0].iters > 30      # more than one restart cycle
        outs.append(x.clone())
    for o in outs[1:]:
        assert torch.equal(o, outs[0])


OPTION_CASES = [
    # (label, shape (n, M, P, sigma, beta, gamma, n_t), options)
    ("M>8 gather kernels", (16, 10, 2, 0.2, 1e-2, 0.0, 1), {}),
    ("M>8 time-dependent", (16, 9, 2, 0.15, 1e-3, 0.0, 3), {}),
    ("unfused Chebyshev", (32, 3, 2, 0.25, 1e-3, 0.0, 1), dict(cheb_steps=12)),
    ("Chebyshev one step", (16, 2, 2, 0.25, 1e-3, 0.0, 1), dict(cheb_steps=1)),
    ("Chebyshev nine steps", (16, 2, 2, 0.25, 1e-3, 0.0, 2), dict(cheb_steps=9)),
    ("smoothing 1/3", (32, 3, 2, 0.25, 1e-3, 0.0, 1), dict(gmg_pre=1, gmg_post=3)),
    ("smoothing 3/1", (32, 3, 2, 0.25, 1e-3, 0.3, 1), dict(gmg_pre=3, gmg_post=1)),
    ("smoothing 4/4", (16, 2, 2, 0.25, 1e-3, 0.0, 2), dict(gmg_pre=4, gmg_post=4)),
    ("truncation r=3", (32, 4, 2, 0.25, 1e-3, 0.0, 1), dict(truncation_r=3)),
    ("coarse-only hierarchy", (8, 2, 2, 0.2, 1e-2, 0.0, 1), {}),
    ("three level kernels above the tail", (256, 2, 1, 0.2, 1e-2, 0.0, 1), {}),
    # the down kernel stores its pre-smoothed iterate and the up kernel reads it:
    # other smoothing degrees on a level above the tail (one pre step, the
    # most pre and post steps, time-dependent columns)
    ("smoothing 1/3 above the tail", (128, 2, 1, 0.25, 1e-3, 0.0, 1), dict(gmg_pre=1, gmg_post=3)),
    ("smoothing 4/1 above the tail", (128, 2, 1, 0.25, 1e-3, 0.3, 1), dict(gmg_pre=4, gmg_post=1)),
    ("smoothing 3/4 above the tail, time", (128, 1, 1, 0.2, 1e-3, 0.0, 2), dict(gmg_pre=3, gmg_post=4)),
    ("exact mean-block solves", (32, 3, 2, 0.25, 1e-3, 0.0, 1), dict(mean_solver=1)),
    ("exact mean-block solves, time", (16, 3, 2, 0.25, 1e-3, 0.0, 3), dict(mean_solver=1)),
    ("exact mass solves", (32, 3, 2, 0.25, 1e-3, 0.3, 1), dict(cheb_steps=0)),
    ("exact mass solves, time", (16, 2, 2, 0.25, 1e-3, 0.3, 3), dict(cheb_steps=0)),
    ("exact solves, two tiles", (128, 2, 2, 0.2, 1e-2, 0.0, 1), dict(cheb_steps=0, mean_solver=1)),
    ("Richardson N=3", (32, 3, 2, 0.25, 1e-3, 0.0, 1), dict(richardson_steps=3)),
    ("Richardson N=2 exact, time, r=2", (16, 3, 2, 0.25, 1e-3, 0.0, 2),
     dict(richardson_steps=2, mean_solver=1, truncation_r=2)),
    ("Richardson M>8, r=4", (16, 10, 2, 0.2, 1e-2, 0.0, 1), dict(richardson_steps=2, truncation_r=4)),
]


@pytest.mark.parametrize("label,shape,opts", OPTION_CASES, ids=[c[0] for c in OPTION_CASES])
def test_option_paths(label, shape, opts):
    """Code paths the default workloads do not take: the gather kernels for
    M > 8, the per-step Chebyshev kernel (more than 9 steps), other smoothing
    degrees (separate kernel instances, in the fused tail and in the level
    kernels above it), intermediate truncation, the hierarchy that is only the
    coarse grid, and several level kernels above the fused tail.  KKT and preconditioner applies against the oracle, then
    the solve (against the direct solution, or the oracle's true residual at
    the large grid)."""
    n, M, P, sigma, beta, gamma, nt = shape
    dev = _dev()
    _say(f"option path {label} {shape} {opts}")
    prob, kw = make_case(n, M, P, sigma, beta, gamma, nt, y0=nt > 1)
    sg = kkt.setup(prob)
    # at 256 x 256 the FP64 residual floor of this system is a few 1e-12
    rtol = 1e-12 if n <= 32 else 1e-10
    # a single Chebyshev step is a weak mass-block preconditioner: more iterations to 1e-12
    max_iter = 3000 if opts.get("cheb_steps", 5) == 1 else 600
    h = _setup([kw], rtol=rtol, max_iter=max_iter, **opts)
    rng = np.random.default_rng(9)
    x = rng.uniform(-1, 1, size=kkt.rhs(sg).size)
    xd = torch.from_numpy(kkt_to_canonical(sg, x)).to(dev)
    yd = torch.full_like(xd, np.nan)          # every output node, ring included, must be written
    h.apply_kkt(xd, yd)
    zd = torch.full_like(xd, np.nan)
    h.precond_apply(xd, zd)
    torch.cuda.synchronize()
    assert ring_is_zero(yd.cpu().numpy(), n) and ring_is_zero(zd.cpu().numpy(), n)
    assert rel_max(canonical_to_kkt(sg, yd.cpu().numpy()), kkt.kkt_apply_matricized(sg, x)) < 1e-12
    inner = precond.make_inner(sg, "exact" if opts.get("mean_solver", 0) == 1 else "gmg",
                               nu_pre=opts.get("gmg_pre", 2), nu_post=opts.get("gmg_post", 2))
    r = opts.get("truncation_r", 0) or M + 1
    ref = precond.precond_apply(sg, x, inner, r, cheb_steps=opts.get("cheb_steps", 5),
                                richardson_steps=opts.get("richardson_steps", 1))
    assert rel_max(canonical_to_kkt(sg, zd.cpu().numpy()), ref) < 1e-12
    sol = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
    rc, info = h.solve(sol)
    assert rc == 0 and info[0].rel_res_true <= rtol, (rc, info[0].rel_res_true)
    xs = canonical_to_kkt(sg, sol.cpu().numpy())
    b = kkt.rhs(sg)
    assert np.linalg.norm(b - kkt.kkt_apply_matricized(sg, xs)) / np.linalg.norm(b) < 10 * rtol
    if n <= 32 and b.size <= 60000:     # the oracle's sparse LU takes minutes above this
        for a, bb in zip(kkt.split(sg, xs), kkt.split(sg, kkt.solve_direct(sg))):
            assert rel_max(a, bb) < 1e-8


HGSOC_CASES = [
    # n, M, P, sigma, beta, gamma, field, options
    (16, 3, 3, 0.3, 1e-2, 0.0, "affine", {}),
    (32, 3, 2, 0.3, 1e-3, 0.5, "affine", dict(truncation_r=3)),
    (16, 2, 2, 0.3, 1e-2, 1.0, "lognormal", {}),
    (16, 3, 2, 0.3, 1e-2, 0.0, "affine", dict(mean_solver=1)),
]

HGSOC_PINT_CASES = [
    # n, M, P, sigma, beta, gamma, n_t, field, options
    (16, 3, 2, 0.3, 1e-2, 0.0, 3, "affine", {}),
    (16, 2, 3, 0.25, 1e-3, 0.5, 4, "affine", dict(truncation_r=2)),
    (16, 2, 2, 0.3, 1e-2, 1.0, 3, "lognormal", dict(mean_solver=1)),
]


def test_hgsoc_batch_equals_alone():
    """hGSoc batches (steady, and time-dependent under Algorithm 4): members
    with different sigma and beta give the iterations and bit-identical
    solutions of their alone solves."""
    dev = _dev()
    sgl = _lib()
    _say("hgsoc batch invariance")
    for nt in (1, 3):
        kws = [make_case(16, 3, 2, sg, b, 0.0, nt, seed=sd, y0=nt > 1)[1]
               for sg, b, sd in ((0.2, 1e-2, 0), (0.3, 1e-3, 1))]
        hb = _setup(kws, precond=sgl.SG_PRECOND_HGSOC, rtol=1e-10, max_iter=600)
        xb = torch.zeros(2 * hb.kkt_elems, dtype=torch.float64, device=dev)
        rc, infos = hb.solve(xb)
        assert rc == 0
        for i, kw in enumerate(kws):
            ha = _setup([kw], precond=sgl.SG_PRECOND_HGSOC, rtol=1e-10, max_iter=600)
            xa = torch.zeros(ha.kkt_elems, dtype=torch.float64, device=dev)
            rca, ia = ha.solve(xa)
            assert rca == 0 and ia[0].iters == infos[i].iters
            assert torch.equal(xa, xb[i * ha.kkt_elems:(i + 1) * ha.kkt_elems])


@pytest.mark.parametrize("case", HGSOC_PINT_CASES)
def test_hgsoc_pint_preconditioner(case):
    """SG_PRECOND_HGSOC on the all-at-once time-dependent system (Algorithm 4:
    Algorithms 2-3 on every time step, with the step's blocks and A-hat_1):
    the preconditioner apply against the oracle's hgsoc_pint at 1e-12 (FP32
    at 1e-5), and a solve within 1e-8 of the direct solution."""
    n, M, P, sigma, beta, gamma, nt, field, opts = case
    dev = _dev()
    _say(f"hgsoc pint {case}")
    sgl = _lib()
    prob, kw = make_case(n, M, P, sigma, beta, gamma, nt, y0=True, field=field)
    sg = kkt.setup(prob)
    h = _setup([kw], precond=sgl.SG_PRECOND_HGSOC, rtol=1e-12, max_iter=800, **opts)
    x = np.random.default_rng(23).uniform(-1, 1, size=kkt.rhs(sg).size)
    xd = torch.from_numpy(kkt_to_canonical(sg, x)).to(dev)
    zd = torch.full_like(xd, np.nan)
    h.precond_apply(xd, zd)
    z32 = torch.full_like(xd, np.nan, dtype=torch.float32)
    h.precond_apply(xd.float(), z32)
    torch.cuda.synchronize()
    pt = precond.PtildeSolve(sg, "cheb", adjoint="schur")
    pt.inner = precond.make_inner(sg, "exact" if opts.get("mean_solver", 0) == 1 else "gmg")
    ref = precond.hgsoc_pint(sg, x, pt, opts.get("truncation_r", 0) or len(sg.G))
    assert rel_max(canonical_to_kkt(sg, zd.cpu().numpy()), ref) < 1e-12
    assert rel_max(canonical_to_kkt(sg, z32.double().cpu().numpy()), ref) < 1e-5
    assert ring_is_zero(zd.cpu().numpy(), n)
    sol = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
    rc, info = h.solve(sol)
    assert rc == 0 and info[0].rel_res_true <= 1e-12
    xs = canonical_to_kkt(sg, sol.cpu().numpy())
    for a, b in zip(kkt.split(sg, xs), kkt.split(sg, kkt.solve_direct(sg))):
        assert rel_max(a, b) < 1e-8


@pytest.mark.parametrize("case", HGSOC_CASES)
def test_hgsoc_preconditioner(case):
    """SG_PRECOND_HGSOC (Algorithms 2-3 with the Schur-type level solves):
    the preconditioner apply against the oracle's hgsoc (same Chebyshev and
    multigrid level solves) at 1e-12, the FP32 apply at 1e-5, and a solve
    within 1e-8 of the direct solution."""
    n, M, P, sigma, beta, gamma, field, opts = case
    dev = _dev()
    _say(f"hgsoc {case}")
    sgl = _lib()
    prob, kw = make_case(n, M, P, sigma, beta, gamma, field=field)
    sg = kkt.setup(prob)
    h = _setup([kw], precond=sgl.SG_PRECOND_HGSOC, rtol=1e-12, max_iter=800, **opts)
    rng = np.random.default_rng(21)
    x = rng.uniform(-1, 1, size=kkt.rhs(sg).size)
    xd = torch.from_numpy(kkt_to_canonical(sg, x)).to(dev)
    zd = torch.full_like(xd, np.nan)
    h.precond_apply(xd, zd)
    z32 = torch.full_like(xd, np.nan, dtype=torch.float32)
    h.precond_apply(xd.float(), z32)
    torch.cuda.synchronize()
    mode = "exact" if opts.get("mean_solver", 0) == 1 else "gmg"
    pt = precond.PtildeSolve(sg, "cheb", adjoint="schur")
    pt.inner = precond.make_inner(sg, mode)
    r = opts.get("truncation_r", 0) or len(sg.G)
    ref = precond.hgsoc(sg, x, pt, r)
    assert rel_max(canonical_to_kkt(sg, zd.cpu().numpy()), ref) < 1e-12
    assert rel_max(canonical_to_kkt(sg, z32.double().cpu().numpy()), ref) < 1e-5
    assert ring_is_zero(zd.cpu().numpy(), n)
    sol = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
    rc, info = h.solve(sol)
    assert rc == 0 and info[0].rel_res_true <= 1e-12
    xs = canonical_to_kkt(sg, sol.cpu().numpy())
    for a, b in zip(kkt.split(sg, xs), kkt.split(sg, kkt.solve_direct(sg))):
        assert rel_max(a, b) < 1e-8


KAPPA_CASES = [
    # n, M, P, beta, gamma, n_t, field seed
    (16, 3, 2, 1e-2, 0.4, 1, 31),
    (32, 2, 3, 1e-3, 0.0, 1, 32),
    (16, 2, 2, 1e-3, 0.3, 3, 33),
    (16, 9, 1, 1e-2, 0.0, 1, 34),        # M > 8: gather kernels
    (16, 9, 1, 1e-2, 0.2, 2, 35),        # M > 8, time-dependent
]


@pytest.mark.parametrize("case", KAPPA_CASES)
def test_explicit_kappa_field(case):
    """A caller-supplied coefficient (sg_problem.kappa) whose modes are not
    symmetric under x <-> y and whose mean is not 1: the library reads the
    per-element modes in [k][ey][ex] order in every kernel (sweeps, mass and
    multigrid constants, gather kernels for M > 8).  Operator, KKT and
    preconditioner applies (full and truncated) against the oracle at 1e-12,
    and the solve against the direct solution at 1e-8."""
    import sg_inputs
    n, M, P, beta, gamma, nt, seed = case
    dev = _dev()
    _say(f"explicit kappa {case}")
    kappa = sg_inputs.field_modes(n, M, seed)
    assert np.max(np.abs(kappa[1] - kappa[1].T)) > 1e-2       # the field really is asymmetric
    prob, kw = make_case(n, M, P, 0.0, beta, gamma, nt, y0=nt > 1, kappa=kappa)
    sg = kkt.setup(prob)
    rng = np.random.default_rng(41)
    X = rng.uniform(-1, 1, size=(max(nt, 1), sg.n_xi, (n + 1) ** 2))
    for r_trunc in (0, 2):
        h = _setup([kw], truncation_r=r_trunc, rtol=1e-12, max_iter=600)
        Xd = torch.from_numpy(X).to(dev)
        Yd = torch.full_like(Xd, np.nan)
        h.apply_operator(Xd, Yd)
        x = rng.uniform(-1, 1, size=kkt.rhs(sg).size)
        xd = torch.from_numpy(kkt_to_canonical(sg, x)).to(dev)
        yd = torch.full_like(xd, np.nan)
        h.apply_kkt(xd, yd)
        zd = torch.full_like(xd, np.nan)
        h.precond_apply(xd, zd)
        torch.cuda.synchronize()
        Y = Yd.cpu().numpy()
        for t in range(max(nt, 1)):
            assert rel_max(fem.extract(Y[t], n), kkt.operator_apply(sg, fem.extract(X[t], n))) < 1e-12
        assert rel_max(canonical_to_kkt(sg, yd.cpu().numpy()), kkt.kkt_matrix(sg) @ x) < 1e-12
        ref = precond.precond_apply(sg, x, precond.make_inner(sg), r_trunc if r_trunc else M + 1)
        assert rel_max(canonical_to_kkt(sg, zd.cpu().numpy()), ref) < 1e-12
        assert ring_is_zero(yd.cpu().numpy(), n) and ring_is_zero(zd.cpu().numpy(), n)
        if r_trunc == 0:
            sol = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
            rc, info = h.solve(sol)
            assert rc == 0 and info[0].rel_res_true <= 1e-12
            xs = canonical_to_kkt(sg, sol.cpu().numpy())
            for a, b in zip(kkt.split(sg, xs), kkt.split(sg, kkt.solve_direct(sg))):
                assert rel_max(a, b) < 1e-8
        h.close()


@pytest.mark.parametrize("precision,max_iter", [(0, 1), (0, 7), (1, 3), (2, 5)])
def test_not_converged_reports_true_residual(precision, max_iter):
    """An iteration budget too small for rtol: sg_solve returns
    SG_NOT_CONVERGED, the member's report says so (status, converged = 0, the
    iterations actually spent), and rel_res_true is the FP64 residual of the
    returned iterate, recomputed here by the oracle."""
    sgl = _lib()
    dev = _dev()
    _say(f"not converged precision={precision} max_iter={max_iter}")
    prob, kw = make_case(16, 3, 2, 0.3, 1e-4, seed=6)
    sg = kkt.setup(prob)
    h = _setup([kw], rtol=1e-10, max_iter=max_iter, precision=precision)
    xd = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
    rc, info = h.solve(xd)
    assert rc == sgl.SG_NOT_CONVERGED
    assert info[0].status == sgl.SG_NOT_CONVERGED and info[0].converged == 0
    assert 1 <= info[0].iters <= max_iter
    x = canonical_to_kkt(sg, xd.cpu().numpy())
    b = kkt.rhs(sg)
    res = np.linalg.norm(b - kkt.kkt_matrix(sg) @ x) / np.linalg.norm(b)
    assert res > 1e-10
    assert abs(info[0].rel_res_true - res) <= 1e-6 * res, (info[0].rel_res_true, res)
