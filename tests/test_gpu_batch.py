"""Batched systems (one launch per phase for all systems): every system of
the batch against the oracle run on that system alone."""
import numpy as np
import pytest

from oracle.ljref import half_pairs_set
from paper_1806_05713_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_05713_amd import lj
    return lj


@pytest.fixture(scope="module")
def ctx(lj):
    c = lj.Context(0, stream=torch.cuda.Stream())
    yield c
    c.close()


def small_batch(count=24, seed=7):
    return synth.batch512(count=count, nmin=256, nmax=2048, seed=seed)


def concat(systems, layout=0):
    pos = np.concatenate([s.pos for s in systems])
    return torch.from_numpy(synth.aos4(pos) if layout == 0 else synth.soa(pos)).to("cuda")


def offsets(systems):
    return np.concatenate([[0], np.cumsum([s.n for s in systems])])


def params(systems):
    n = np.array([s.n for s in systems])
    box = np.array([s.box for s in systems])
    rc = np.array([s.rc for s in systems])
    return n, box, rc


def canon(ij):
    a = np.sort(ij.astype(np.int64), axis=1)
    return a[np.lexsort((a[:, 1], a[:, 0]))]


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("build_lanes", [0, 4])
def test_batch_pairs_and_forces(lj, ctx, oracle, kind, layout, build_lanes):
    systems = small_batch()
    off = offsets(systems)
    n, box, rc = params(systems)
    pos = concat(systems, layout)
    torch.cuda.synchronize()
    ctx.tune_set(lj.LJ_TUNE_BUILD_LANES, build_lanes)
    try:
        with torch.cuda.stream(ctx.stream):
            nl = lj.lj_build_neighbors_batch(ctx, pos, n, box, rc, 0.3, kind=kind)
    finally:
        ctx.tune_set(lj.LJ_TUNE_BUILD_LANES, 0)
    with torch.cuda.stream(ctx.stream):
        ones = np.ones(len(systems))
        F, E, W, C = lj.lj_forces_batch(ctx, pos, nl, ones, ones, rc)
        ctx.sync()
    torch.cuda.synchronize()
    ij = nl.pairs().astype(np.int64)
    sys_of = np.searchsorted(off, ij[:, 0], side="right") - 1
    assert np.all(sys_of == np.searchsorted(off, ij[:, 1], side="right") - 1)
    f = F.cpu().numpy()
    f = f[:, :3] if layout == 0 else f.T
    E, W, C = E.cpu().numpy(), W.cpu().numpy(), C.cpu().numpy()
    for s, sy in enumerate(systems):
        rp, col = oracle.cell_pairs(sy.pos, sy.box, sy.rc + sy.skin)
        ref = half_pairs_set(rp, col)
        mine = ij[sys_of == s] - off[s]
        if kind == 1:
            mine = mine[mine[:, 0] < mine[:, 1]]
        assert np.array_equal(canon(mine), ref), f"system {s}"
        Fr, Er, Wr, nr = oracle.forces(sy.pos, sy.box, 1.0, 1.0, sy.rc, rp, col)
        scale = np.abs(Fr).max()
        assert np.abs(f[off[s]:off[s + 1]] - Fr).max() <= 1e-10 * scale, f"system {s}"
        assert abs(E[s] - Er) <= 1e-12 * abs(Er)
        assert abs(W[s] - Wr) <= 1e-12 * abs(Wr)
        assert C[s] == nr
        n_s, max_row, entries, cap = nl.sys_info(s)
        assert n_s == sy.n and max_row <= cap
        assert entries == (1 if kind == 0 else 2) * ref.shape[0]


@pytest.mark.parametrize("layout", [0, 1])
def test_batch_mixed_forces(lj, ctx, oracle, layout):
    """Mixed precision over a batch: each system's fixed-point unit and
    cutoff band come from its own box and rc; every system's pair count is
    the oracle's exactly and its forces are within 1e-5 of the scale."""
    systems = small_batch(count=12, seed=31)
    off = offsets(systems)
    n, box, rc = params(systems)
    pos = concat(systems, layout)
    torch.cuda.synchronize()
    with torch.cuda.stream(ctx.stream):
        nl = lj.lj_build_neighbors_batch(ctx, pos, n, box, rc, 0.3, kind=1)
        ones = np.ones(len(systems))
        F, E, W, C = lj.lj_forces_batch(ctx, pos, nl, ones, ones, rc, precision=lj.LJ_MIXED)
        ctx.sync()
    torch.cuda.synchronize()
    f = F.cpu().numpy()
    f = f[:, :3] if layout == 0 else f.T
    E, W, C = E.cpu().numpy(), W.cpu().numpy(), C.cpu().numpy()
    for s, sy in enumerate(systems):
        rp, col = oracle.cell_pairs(sy.pos, sy.box, sy.rc + sy.skin)
        Fr, Er, Wr, nr = oracle.forces(sy.pos, sy.box, 1.0, 1.0, sy.rc, rp, col)
        scale = np.abs(Fr).max()
        assert np.abs(f[off[s]:off[s + 1]] - Fr).max() <= 1e-5 * scale, f"system {s}"
        # FP32 pair terms over a few hundred atoms: less averaging than at 4k
        assert abs(E[s] - Er) <= 5e-6 * abs(Er), f"system {s}"
        assert abs(W[s] - Wr) <= 5e-6 * abs(Wr), f"system {s}"
        assert C[s] == nr, f"system {s}"
    nl.free()


def test_batch_two_level_reduction(lj, ctx, oracle):
    """One row per slice (64 lanes per row): the 19,652-atom system has 4,928
    force blocks, so every system's energy, virial and pair count are summed
    in two levels of 2 spans; the small systems' spans are short or empty."""
    systems = [synth.small_fcc(17, 0.9, 0.05, 3, rc=2.5)] + small_batch(count=5, seed=21)
    off = offsets(systems)
    n, box, rc = params(systems)
    pos = concat(systems)
    torch.cuda.synchronize()
    with torch.cuda.stream(ctx.stream):
        nl = lj.lj_build_neighbors_batch(ctx, pos, n, box, rc, 0.3, kind=1, lanes=64)
        ones = np.ones(len(systems))
        F, E, W, C = lj.lj_forces_batch(ctx, pos, nl, ones, ones, rc)
        ctx.sync()
    torch.cuda.synchronize()
    assert nl.info().lanes == 64
    f = F.cpu().numpy()[:, :3]
    E, W, C = E.cpu().numpy(), W.cpu().numpy(), C.cpu().numpy()
    for s, sy in enumerate(systems):
        rp, col = oracle.cell_pairs(sy.pos, sy.box, sy.rc + sy.skin)
        Fr, Er, Wr, nr = oracle.forces(sy.pos, sy.box, 1.0, 1.0, sy.rc, rp, col)
        scale = np.abs(Fr).max()
        assert np.abs(f[off[s]:off[s + 1]] - Fr).max() <= 1e-10 * scale, f"system {s}"
        assert abs(E[s] - Er) <= 1e-12 * abs(Er), f"system {s}"
        assert abs(W[s] - Wr) <= 1e-12 * abs(Wr), f"system {s}"
        assert C[s] == nr, f"system {s}"
    nl.free()


def run_batch_nve(lj, ctx, systems, dt, nsteps, every, use_graph, precision=0):
    n, box, rc = params(systems)
    pos = concat(systems)
    vel = torch.from_numpy(synth.aos4(np.concatenate([s.vel for s in systems]))).to("cuda")
    force = torch.zeros_like(pos)
    torch.cuda.synchronize()
    with torch.cuda.stream(ctx.stream):
        nl = lj.lj_build_neighbors_batch(ctx, pos, n, box, rc, 0.3, kind=1)
        ones = np.ones(len(systems))
        nve = lj.NVE(ctx, pos, vel, force, None, ones, ones, rc, nl, dt, every, precision,
                     log_rows=nsteps + 1, batch=True)
        nve.init()
        nve.run(nsteps, use_graph=use_graph)
        stale = False
        try:
            ctx.sync()
        except lj.LJError as e:      # a fixed cadence whose lists went stale: reported
            if e.status != lj.LJ_E_STALE:
                raise
            stale = True
    torch.cuda.synchronize()
    out = (pos.cpu().numpy()[:, :3].copy(), vel.cpu().numpy()[:, :3].copy(),
           nve.log.cpu().numpy().copy(), stale)
    nve.free()
    nl.free()
    return out


@pytest.mark.parametrize("every", [10, 0])
def test_batch_nve_matches_oracle(lj, ctx, oracle, every):
    """Each system against its own oracle run.  At a fixed cadence the GPU
    reports a stale list exactly when some system's oracle log shows an atom
    moved more than skin/2 at a step between builds; with the displacement
    rule (every = 0) a step rebuilds every system when any needs it, and each
    system's pairs inside rc are still the oracle's at every step."""
    systems = small_batch(count=10, seed=11)
    off = offsets(systems)
    p, v, log, stale = run_batch_nve(lj, ctx, systems, 0.005, 25, every, use_graph=False)
    any_beyond = False
    for s, sy in enumerate(systems):
        pr, vr, _, lr = oracle.nve(sy.pos, sy.vel, sy.box, 1.0, 1.0, sy.rc, sy.skin, 0.005, 25,
                                   every)
        d = p[off[s]:off[s + 1]] - pr
        d -= sy.box[0] * np.round(d / sy.box[0])
        assert np.abs(d).max() < 1e-9, f"system {s}"
        assert np.abs(v[off[s]:off[s + 1]] - vr).max() < 1e-8
        np.testing.assert_allclose(log[:, s, 0], lr[:, 0], rtol=1e-9)
        np.testing.assert_allclose(log[:, s, 1], lr[:, 1], rtol=1e-9)
        np.testing.assert_allclose(log[:, s, 2], lr[:, 2], rtol=1e-9)
        assert np.array_equal(log[:, s, 4], lr[:, 4])
        if every:
            assert np.array_equal(log[:, s, 5], lr[:, 5])
            np.testing.assert_allclose(log[:, s, 3], lr[:, 3], rtol=1e-6, atol=1e-12)
            between = lr[:, 5] == 0.0
            any_beyond = any_beyond or bool(np.any(lr[between, 3] > 0.5 * sy.skin))
    if every:
        assert stale == any_beyond
    else:
        assert not stale
        # every system rebuilt together, at least once
        assert np.all(log[:, :, 5] == log[:, :1, 5]) and log[1:, 0, 5].sum() >= 1


def test_batch_nve_graph_equals_eager(lj, ctx):
    systems = small_batch(count=16, seed=12)
    a = run_batch_nve(lj, ctx, systems, 0.005, 30, 10, use_graph=False)
    b = run_batch_nve(lj, ctx, systems, 0.005, 30, 10, use_graph=True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_batch512_full_size(lj, ctx, oracle):
    """The 512-system batch (about 4.3M atoms): exact pairs and forces for a
    sample of systems, zero net force in every system."""
    systems = synth.batch512()
    off = offsets(systems)
    n, box, rc = params(systems)
    pos = concat(systems)
    torch.cuda.synchronize()
    with torch.cuda.stream(ctx.stream):
        nl = lj.lj_build_neighbors_batch(ctx, pos, n, box, rc, 0.3, kind=1)
        ones = np.ones(len(systems))
        F, E, W, C = lj.lj_forces_batch(ctx, pos, nl, ones, ones, rc)
        ctx.sync()
    torch.cuda.synchronize()
    f = F.cpu().numpy()[:, :3]
    E = E.cpu().numpy()
    for s in range(len(systems)):
        net = np.abs(f[off[s]:off[s + 1]].sum(axis=0)).max()
        assert net <= 1e-10 * max(np.abs(f[off[s]:off[s + 1]]).max(), 24.0) * np.sqrt(systems[s].n)
    rng = np.random.Generator(np.random.PCG64(3))
    for s in sorted(rng.choice(len(systems), size=6, replace=False)) + [int(np.argmax(n)), int(np.argmin(n))]:
        sy = systems[s]
        rp, col = oracle.cell_pairs(sy.pos, sy.box, sy.rc + sy.skin)
        Fr, Er, Wr, nr = oracle.forces(sy.pos, sy.box, 1.0, 1.0, sy.rc, rp, col)
        assert np.abs(f[off[s]:off[s + 1]] - Fr).max() <= 1e-10 * max(np.abs(Fr).max(), 24.0)
        assert abs(E[s] - Er) <= 1e-12 * abs(Er)
        assert nl.sys_info(s)[2] == 2 * col.size
