"""GPU tests of the batched path: uneven cases advanced together must reproduce each
case advanced alone with the same tile (the single-case path is itself checked against
the oracle), the hipGraph replay must equal eager launches, and the autotuner and the
slot balancing must leave the state untouched."""
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _v():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_10899_amd import vclb
    return vclb


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_batch(storage="fp64", n=6, seed=7):
    cases, _ = W.batch_cases(n_cases=n, seed=seed, storage=storage, side_lo=40, side_hi=150)
    return cases


@pytest.mark.parametrize("storage,flat_pct,bx", [("fp64", 0, 64), ("fp64", 90, 64), ("fp64", 101, 64),
                                                 ("fp16s", 90, 64), ("fp32", 101, 64), ("fp64", 100, 512),
                                                 ("fp32", 0, 512), ("fp32", 101, 1024), ("fp16s", 0, 1024)])
def test_batch_matches_cases_run_alone(storage, flat_pct, bx):
    """Column strips (flat_pct 0), flattened bands (101), the mixes (90, 100), 64, 512 and
    1024 lanes."""
    v = _v()
    cases = small_batch(storage)
    say("case: batch of", [(p.nx, p.ny, p.wall_y) for p, _, _ in cases], storage, "flat_pct", flat_pct, "bx", bx)
    b = v.Batch([p for p, _, _ in cases])
    b.set_tile(bx, 16)
    b.set_schedule(flat_pct)
    assert b.schedule() == flat_pct
    for c, (p, phi0, u0) in zip(b.cases, cases):
        c.init(phi0, u0)
    b.step(25)
    for k, (p, phi0, u0) in enumerate(cases):
        alone = v.Case(p, tile=(64, 16)).init(phi0, u0)
        alone.step(25)
        ga, fa, Ja = alone.get_state()
        gb, fb, Jb = b.cases[k].get_state()
        err = max(np.max(np.abs(ga - gb)), np.max(np.abs(fa - fb)), np.max(np.abs(Ja - Jb)))
        say(f"  case {k} {p.nx}x{p.ny}: max |batch - alone| = {err:.3e}")
        assert err <= (1e-13 if storage == "fp64" else 1e-5), k
        ha, hb = alone.history(0, 25), b.cases[k].history(0, 25)
        assert np.allclose(ha["sum_phi"], hb["sum_phi"], rtol=1e-12 if storage == "fp64" else 1e-6)


@pytest.mark.parametrize("flat_pct", [0, 101])
def test_batch_with_custom_rates_matches_cases_run_alone(flat_pct):
    """A case with rates off their defaults switches the whole batch to the general-rate
    kernel; every case must still reproduce its own run (which picks per case)."""
    v = _v()
    cases = small_batch("fp64", n=4, seed=9)
    p0, phi0, u0 = cases[1]
    cases[1] = (p0.replace(s_g=(0, 1.3, 1.1, 0, 0, 0, 0, 1.7, 0.9), s_f=(1.2, 1.4, 1.6, 0.8, 1.5, 0.8, 1.5, 0, 0)),
                phi0, u0)
    say("case: batch with one custom-rate case, flat_pct", flat_pct)
    b = v.Batch([p for p, _, _ in cases])
    b.set_tile(256, 16)
    b.set_schedule(flat_pct)
    for c, (p, phi0, u0) in zip(b.cases, cases):
        c.init(phi0, u0)
    b.step(20)
    for k, (p, phi0, u0) in enumerate(cases):
        alone = v.Case(p, tile=(64, 16)).init(phi0, u0)
        alone.step(20)
        err = max(np.max(np.abs(a_ - b_)) for a_, b_ in zip(alone.get_state(), b.cases[k].get_state()))
        say(f"  case {k}: max |batch - alone| = {err:.3e}")
        assert err <= 1e-13, k


@pytest.mark.parametrize("flat_pct,bx", [(101, 512), (0, 256), (101, 64)])
def test_batch_extreme_sizes_matches_cases_run_alone(flat_pct, bx):
    """One large case among tiny ones: the run partition splits the large case over
    many workgroups (bands of a few rows) and packs the tiny ones together, and a case
    one node wide or two rows high still steps exactly as alone."""
    v = _v()
    specs = [(300, 260, False), (1, 40, False), (3, 130, True), (8, 8, False), (70, 2, True), (5, 9, False)]
    cases = []
    for nx, ny, wall in specs:
        p = W.CaseParams(nx=nx, ny=ny, rho_light=0.2, wall_y=wall,
                         wall_u_bottom=(-0.02, 0.0, 0.0) if wall else (0.0, 0.0, 0.0),
                         wall_u_top=(0.02, 0.0, 0.0) if wall else (0.0, 0.0, 0.0))
        R = max(1.5, 0.3 * min(nx, ny))
        cases.append((p, W.drops_phi(p, [((nx - 1) / 2.0, (ny - 1) / 2.0, 0.0, R)]),
                      W.couette_u(p) if wall else None))
    say("case: extreme sizes", specs, "flat_pct", flat_pct, "bx", bx)
    b = v.Batch([p for p, _, _ in cases])
    b.set_tile(bx, 1024)
    b.set_schedule(flat_pct)
    for c, (p, phi0, u0) in zip(b.cases, cases):
        c.init(phi0, u0)
    b.step(12)
    for k, (p, phi0, u0) in enumerate(cases):
        alone = v.Case(p, tile=(64, 16)).init(phi0, u0)
        alone.step(12)
        err = max(np.max(np.abs(a_ - b_)) for a_, b_ in zip(alone.get_state(), b.cases[k].get_state()))
        say(f"  case {k} {p.nx}x{p.ny}: max |batch - alone| = {err:.3e}")
        assert err <= 1e-13, k
        ha, hb = alone.history(0, 12), b.cases[k].history(0, 12)
        assert np.allclose(ha["sum_phi"], hb["sum_phi"], rtol=1e-12)


def test_batch_graph_equals_eager_and_history():
    v = _v()
    cases = small_batch("fp32", n=5, seed=3)
    runs = []
    for graph in (True, False):
        b = v.Batch([p for p, _, _ in cases])
        for c, (p, phi0, u0) in zip(b.cases, cases):
            c.init(phi0, u0)
        b.step(7, graph=graph)
        b.step(6, graph=graph)
        runs.append((b, [c.get_state() for c in b.cases]))
    for k in range(len(cases)):
        for a, c in zip(runs[0][1][k], runs[1][1][k]):
            assert np.array_equal(a, c), k
    b = runs[0][0]
    for k, c in enumerate(b.cases):
        assert c.time() == 13
        h = c.history(0, 13)
        assert np.all(h["step"][:, 0] == np.arange(13))
        r = c.reduce()
        assert abs(r["sum_phi"][0] - h["sum_phi"][-1, 0]) <= 1e-5 * abs(r["sum_phi"][0])


def test_batch_reduce_and_history_match_each_case():
    """The batch-level reductions equal each case's own reduce() and history()."""
    v = _v()
    cases = small_batch("fp64", n=5, seed=5)
    b = v.Batch([p for p, _, _ in cases])
    for c, (p, phi0, u0) in zip(b.cases, cases):
        c.init(phi0, u0)
    b.step(9)
    r = b.reduce()
    h = b.history(2, 7)
    assert r["rc"] == v.VCLB_OK
    assert r["sum_phi"].shape == (len(cases), v.MAX_LABELS)
    assert h["sum_phi"].shape == (7, len(cases), v.MAX_LABELS)
    for k, c in enumerate(b.cases):
        nl = c.nlabels
        rk = c.reduce()
        hk = c.history(2, 7)
        for f in ("sum_phi", "count_half", "sum_phi_d", "sum_phi_dd"):
            assert np.array_equal(r[f][k, :nl], rk[f]), (k, f)
            assert np.array_equal(h[f][:, k, :nl], hk[f]), (k, f)
        assert np.all(r["sum_phi"][k, nl:] == 0.0)
        assert np.all(h["step"][:, k, :] == np.arange(2, 9)[:, None])
    assert b.history(0, 9)["sum_phi"].shape[0] == 9
    with pytest.raises(v.VclbError):
        b.history(5, 10)                       # steps 9..14 were never taken


def test_batch_autotune_restores_state_and_uses_cache(tmp_path):
    v = _v()
    cases = small_batch("fp32", n=4, seed=11)
    b = v.Batch([p for p, _, _ in cases])
    for c, (p, phi0, u0) in zip(b.cases, cases):
        c.init(phi0, u0)
    b.step(3)
    before = [c.get_state() for c in b.cases]
    cache = str(tmp_path / "tiles.jsonl")
    tile = b.autotune(cache, steps=2)
    say("  autotuned tile", tile)
    after = [c.get_state() for c in b.cases]
    for x, y in zip(before, after):
        for a, c in zip(x, y):
            assert np.array_equal(a, c)
    assert all(c.time() == 3 for c in b.cases)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"bx"' in lines[0]
    b.set_tile(64, 64)
    assert b.autotune(cache, steps=2)[:2] == tile[:2]        # read back from the cache
    assert len(open(cache).read().strip().splitlines()) == 1


@pytest.mark.parametrize("flat_pct", [101, 0])
def test_batch_1024_lanes_with_wide_and_tiny_cases(flat_pct):
    """1024-lane workgroups (FP32) over a case wider than one chunk (1100 columns: the
    four-slot FIFO in bands, two strips of which one ragged) beside tiny ones."""
    v = _v()
    specs = [(1100, 40, False), (1, 40, False), (3, 130, True), (600, 30, True), (70, 2, True)]
    cases = []
    for nx, ny, wall in specs:
        p = W.CaseParams(nx=nx, ny=ny, rho_light=0.2, wall_y=wall, storage="fp32",
                         wall_u_bottom=(-0.02, 0.0, 0.0) if wall else (0.0, 0.0, 0.0),
                         wall_u_top=(0.02, 0.0, 0.0) if wall else (0.0, 0.0, 0.0))
        R = max(1.5, 0.3 * min(nx, ny))
        cases.append((p, W.drops_phi(p, [((nx - 1) / 2.0, (ny - 1) / 2.0, 0.0, R)]),
                      W.couette_u(p) if wall else None))
    say("case: 1024 lanes, wide and tiny, fp32", specs, "flat_pct", flat_pct)
    b = v.Batch([p for p, _, _ in cases]).init([(phi0, u0) for _, phi0, u0 in cases])
    b.set_tile(1024, 1024)
    b.set_schedule(flat_pct)
    b.step(12)
    for k, (p, phi0, u0) in enumerate(cases):
        alone = v.Case(p, tile=(64, 16)).init(phi0, u0)
        alone.step(12)
        err = max(np.max(np.abs(a_ - b_)) for a_, b_ in zip(alone.get_state(), b.cases[k].get_state()))
        say(f"  case {k} {p.nx}x{p.ny}: max |batch - alone| = {err:.3e}")
        assert err == 0.0, k        # the same node arithmetic in both marches: bit for bit


@pytest.mark.parametrize("storage,bx", [("fp32", 1024), ("fp64", 512)])
def test_band_lag_and_ring_boundaries(storage, bx):
    """Widths at the band march's limits for bx lanes: the one-chunk lag holds up to
    nx + 1 = bx (bx - 1 columns), one more column needs the three-chunk lag; the ring grows
    past 4096 entries at 512 columns with 1024 lanes; narrow rows cross many row starts
    per chunk.  Every case, marched in bands beside the others (flat_pct 101), equals the
    same case stepped alone in strips bit for bit."""
    v = _v()
    widths = [bx - 1, bx, bx + 1, bx // 2 - 1, bx // 2, 65, 64, 63, 5]
    cases = []
    for k, nx in enumerate(widths):
        ny = 5 + k % 3
        wall = k % 2 == 1
        p = W.CaseParams(nx=nx, ny=ny, rho_light=0.25, wall_y=wall, storage=storage,
                         wall_u_bottom=(-0.02, 0.0, 0.0) if wall else (0.0, 0.0, 0.0),
                         wall_u_top=(0.02, 0.0, 0.0) if wall else (0.0, 0.0, 0.0))
        cx, cy = nx * 0.37 + 0.21, ny * 0.5 + 0.13
        cases.append((p, W.drops_phi(p, [(cx, cy, 0.0, max(1.5, 0.4 * min(nx, ny)))]), None))
    say("case: band lag and ring boundaries", storage, bx, widths)
    b = v.Batch([p for p, _, _ in cases]).init([(phi0, u0) for _, phi0, u0 in cases])
    b.set_tile(bx, 1024)
    b.set_schedule(101)
    b.step(10)
    for k, (p, phi0, u0) in enumerate(cases):
        alone = v.Case(p, tile=(64, 16)).init(phi0, u0)
        alone.step(10)
        err = max(np.max(np.abs(a_ - b_)) for a_, b_ in zip(alone.get_state(), b.cases[k].get_state()))
        say(f"  case {k} {p.nx}x{p.ny}: max |batch - alone| = {err:.3e}")
        assert err == 0.0, k


def test_batch_rejects_1024_lanes_in_fp64():
    v = _v()
    b = v.Batch([p for p, _, _ in small_batch("fp64", n=2)])
    with pytest.raises(v.VclbError):
        b.set_tile(1024, 16)
    assert b.tile()[0] == 512                              # the shape in force is kept


@pytest.mark.parametrize("storage,flat_pct,bx", [("fp32", 101, 64), ("fp64", 0, 256), ("fp16s", 100, 1024)])
def test_batch_any_slot_weights_give_the_same_states(storage, flat_pct, bx):
    """Runs cut with arbitrary, even extreme, slot weights still cover every row of every
    case exactly once: the states match the equal cut bit for bit."""
    v = _v()
    cases = small_batch(storage, n=8, seed=9)
    say("case: slot weights", storage, flat_pct, bx, [(p.nx, p.ny) for p, _, _ in cases])

    def make():
        b = v.Batch([p for p, _, _ in cases]).init([(phi0, u0) for _, phi0, u0 in cases])
        b.set_tile(bx, 16)
        b.set_schedule(flat_pct)
        return b

    ref = make()
    ref.step(12)
    n = len(ref.weights())
    assert n == ref.tile()[2] and np.all(ref.weights() == 1.0)
    rng = np.random.Generator(np.random.PCG64(5))
    patterns = {"log-uniform": np.exp(rng.uniform(np.log(0.01), np.log(100.0), n)),
                "one heavy slot": np.where(np.arange(n) == 3, 1e3, 1e-3)}
    for name, w in patterns.items():
        b = make()
        b.set_weights(w)
        got = b.weights()
        assert np.allclose(got, w * n / w.sum(), rtol=1e-12)
        b.step(12)
        for k in range(len(cases)):
            for a, c in zip(ref.cases[k].get_state(), b.cases[k].get_state()):
                assert np.array_equal(a, c), (name, k)
        assert np.allclose(ref.history(0, 12)["sum_phi"], b.history(0, 12)["sum_phi"], rtol=1e-12, atol=0.0)
        b.set_weights([])
        assert np.all(b.weights() == 1.0)
        with pytest.raises(v.VclbError):
            b.set_weights(np.ones(n + 1))               # one weight per slot
        with pytest.raises(v.VclbError):
            b.set_weights(np.zeros(n))                  # outside [1e-3, 1e3]


def test_batch_init_equals_per_case_init():
    """vclb_batch_init gives every case the state vclb_case_init gives it, bit for bit."""
    v = _v()
    cases = small_batch("fp32", n=5, seed=3)
    say("case: batch init of", [(p.nx, p.ny, p.wall_y, u0 is not None) for p, _, u0 in cases])
    one = v.Batch([p for p, _, _ in cases])
    for c, (p, phi0, u0) in zip(one.cases, cases):
        c.init(phi0, u0)
    all_ = v.Batch([p for p, _, _ in cases]).init([(phi0, u0) for _, phi0, u0 in cases])
    for k in range(len(cases)):
        assert all_.cases[k].time() == 0
        for a, b in zip(one.cases[k].get_state(), all_.cases[k].get_state()):
            assert np.array_equal(a, b), k
    one.step(5)
    all_.step(5)
    for k in range(len(cases)):
        for a, b in zip(one.cases[k].get_state(), all_.cases[k].get_state()):
            assert np.array_equal(a, b), k
    with pytest.raises(v.VclbError):
        all_.init([(cases[0][1], None)])                     # one pair per case
    bad = cases[1][1].copy()
    bad.flat[7] = np.nan
    with pytest.raises(v.VclbError):
        all_.init([(phi0, u0) if k != 1 else (bad, u0) for k, (_, phi0, u0) in enumerate(cases)])


@pytest.mark.parametrize("storage,flat_pct,bx", [("fp64", 101, 64), ("fp16s", 0, 256), ("fp32", 100, 512)])
def test_batch_balance_restores_state_and_keeps_results(storage, flat_pct, bx):
    """Slot balancing times launches on the state and restores it; stepping with the re-cut
    runs gives bit-identical states to stepping with runs of equal modelled cost (each
    node's update does not depend on the cut), and the reductions agree to rounding."""
    v = _v()
    cases = small_batch(storage, n=8, seed=5)
    say("case: balance", storage, "flat_pct", flat_pct, "bx", bx, [(p.nx, p.ny) for p, _, _ in cases])

    def make():
        b = v.Batch([p for p, _, _ in cases])
        b.set_tile(bx, 16)
        b.set_schedule(flat_pct)
        for c, (p, phi0, u0) in zip(b.cases, cases):
            c.init(phi0, u0)
        return b

    plain, tuned = make(), make()
    plain.step(3)
    tuned.step(3)
    before = [c.get_state() for c in tuned.cases]
    gain = tuned.balance(rounds=3, steps=2)
    say(f"  slowest slot before / after: {gain:.3f}")
    assert gain >= 1.0
    for x, c in zip(before, tuned.cases):
        for a, y in zip(x, c.get_state()):
            assert np.array_equal(a, y)
    assert all(c.time() == 3 for c in tuned.cases)
    assert tuned.tile()[:2] == (bx, 16) and tuned.schedule() == flat_pct
    plain.step(20)
    tuned.step(20)
    for k in range(len(cases)):
        for a, y in zip(plain.cases[k].get_state(), tuned.cases[k].get_state()):
            assert np.array_equal(a, y), k
    hp, ht = plain.history(3, 20), tuned.history(3, 20)
    assert np.allclose(hp["sum_phi"], ht["sum_phi"], rtol=1e-12, atol=0.0)
    with pytest.raises(v.VclbError):
        tuned.balance(rounds=0)


# --------------------------------------------------------------------------- full size
def _sample(cases):
    """Indices of a few cases that span the batch: largest, smallest, widest, narrowest,
    first shear (walls) and first periodic case."""
    n = [p.nx * p.ny for p, _, _ in cases]
    idx = {int(np.argmax(n)), int(np.argmin(n)), int(np.argmax([p.nx for p, _, _ in cases])),
           int(np.argmin([p.nx for p, _, _ in cases]))}
    idx.add(next(k for k, (p, _, _) in enumerate(cases) if p.wall_y))
    idx.add(next(k for k, (p, _, _) in enumerate(cases) if not p.wall_y))
    return sorted(idx)


# every launch shape the benchmark may time the batch in (bench.BATCH_SHAPES): 512-lane
# workgroups with whole-case items (ty 1024) or items of about 16k nodes (ty 64), with
# bands for the cases that fit the two-slot FIFO and strips for the wider ones
# (flat_pct 100) or bands for every case (101, the four-slot FIFO kernel); and 1024-lane
# workgroups (FP32, FP16S), which fit every case's padded row in one chunk.
import bench  # noqa: E402
FULL_SHAPES = list(bench.BATCH_SHAPES)


def _full_batch(v, storage, bx, ty, flat_pct):
    cases, _ = W.batch_cases(512, storage=storage)
    b = v.Batch([p for p, _, _ in cases])
    b.set_tile(bx, ty)
    b.set_schedule(flat_pct)
    return cases, b


@pytest.mark.parametrize("bx,ty,flat_pct", FULL_SHAPES[:2])
def test_full_batch_fp64_sampled_cases_match_oracle(bx, ty, flat_pct):
    """All 512 cases (24.4 M nodes) in the benchmark's launch configuration; sampled cases
    start from the oracle's exact state and, after one batched step, match the oracle's
    step node by node within the rounding bound of the one-step parity tests."""
    v = _v()
    from oracle.model import Model
    from test_gpu_parity import normal_conditioning
    cases, b = _full_batch(v, "fp64", bx, ty, flat_pct)
    idx = _sample(cases)
    say(f"case: full batch fp64, bx {bx}, ty {ty}, flat_pct {flat_pct}, sampled cases", [(k, cases[k][0].nx, cases[k][0].ny, cases[k][0].wall_y) for k in idx])
    models = {}
    for k, (c, (p, phi0, u0)) in enumerate(zip(b.cases, cases)):
        if k in idx:
            m = Model(p).init(phi0, u0)
            c.set_state(m.g, m.f, m.Jprev, m.t)
            models[k] = (m, normal_conditioning(m, m.fields()))
        else:
            c.init(phi0, u0)
    say(f"  slot balancing (as the benchmark does): gain {b.balance(rounds=3, steps=3):.3f}")
    b.step(1)
    for k in idx:
        m, cond = models[k]
        m.step(1)
        g, f, J = b.cases[k].get_state()
        tol = 1e-13 + 2.0 * cond
        ratio = max(float(np.max(np.abs(g - m.g) / tol[None])), float(np.max(np.abs(f - m.f) / tol[None])),
                    float(np.max(np.abs(J - m.Jprev))) / 1e-13)
        say(f"  case {k}: error / bound {ratio:.3f}")
        assert ratio <= 1.0, k


# per storage: unit round-off of its arithmetic or storage, absolute floor of the
# population bound, bounds on |d phi| and |d u| after one step, volume drift bound
REDUCED = {"fp32": (6e-8, 1e-6, 1e-6, 1e-6, 1e-6), "fp16s": (4.9e-4, 5e-5, 1e-4, 5e-5, 1e-4)}


@pytest.mark.parametrize("bx,ty,flat_pct", FULL_SHAPES)
@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_full_batch_reduced_precision_volume_and_sampled_fields(storage, bx, ty, flat_pct):
    """FP32 and FP16S storage at full size in the benchmark's launch configuration: every
    case keeps its volume (to 1e-6 in FP32, 1e-4 in FP16S) over 20 steps, and sampled
    cases match the FP64 oracle's first step to the storage's rounding (phi, u and the
    populations)."""
    v = _v()
    from oracle.model import Model
    from test_gpu_parity import normal_conditioning
    eps, floor, tol_phi, tol_u, tol_drift = REDUCED[storage]
    cases, b = _full_batch(v, storage, bx, ty, flat_pct)
    idx = _sample(cases)
    say(f"case: full batch {storage}, bx {bx}, ty {ty}, flat_pct {flat_pct}, sampled cases", idx)
    for c, (p, phi0, u0) in zip(b.cases, cases):
        c.init(phi0, u0)
    say(f"  slot balancing (as the benchmark does): gain {b.balance(rounds=3, steps=3):.3f}")
    v0 = b.reduce()["sum_phi"][:, 0]
    b.step(1)
    for k in idx:
        p, phi0, u0 = cases[k]
        m = Model(p.replace(storage="fp64")).init(phi0, u0)
        cond = normal_conditioning(m, m.fields(), eps=eps)
        m.step(1)
        g, f, J = b.cases[k].get_state()
        tol = floor + 2.0 * cond
        ratio = max(float(np.max(np.abs(g - m.g) / tol[None])), float(np.max(np.abs(f - m.f) / tol[None])))
        F = b.cases[k].observe()
        Fo = m.fields()
        dphi = float(np.max(np.abs(F["phi"] - Fo["phi"])))
        du = float(np.max(np.abs(F["u"] - Fo["u"])))
        say(f"  case {k}: populations error / bound {ratio:.3f}, |dphi| {dphi:.2e}, |du| {du:.2e}")
        assert ratio <= 1.0 and dphi <= tol_phi and du <= tol_u, k
    b.step(19)
    v1 = b.reduce()["sum_phi"][:, 0]
    drift = float(np.max(np.abs(v1 - v0) / np.abs(v0)))
    say(f"  max relative volume drift over 20 steps, all 512 cases: {drift:.2e}")
    assert drift <= tol_drift


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_full_batch_keeps_every_volume_over_2000_steps(storage):
    """All 512 cases over the workload's full 2000 steps in the benchmark's launch shape:
    every case keeps sum(phi) to 1e-6.  With 2-byte storage this holds because the
    writer phi absorbs the rounding of the stored deviations; without that, a small
    drop at rest drifted steadily to 1.4e-4."""
    v = _v()
    cases, _ = W.batch_cases(512, storage=storage)
    say(f"case: full batch {storage}, 2000 steps, volume drift")
    b = v.Batch([p for p, _, _ in cases]).init([(phi0, u0) for _, phi0, u0 in cases])
    b.set_tile(1024 if storage == "fp32" else 512, 1024)
    b.set_schedule(101)
    b.set_reduce_every(0)
    v0 = b.reduce()["sum_phi"][:, 0]
    b.step(2000)
    d = np.abs(b.reduce()["sum_phi"][:, 0] - v0) / np.abs(v0)
    say(f"  max relative drift {d.max():.2e}, median {np.median(d):.2e}")
    assert d.max() <= 1e-6                           # measured: 1.0e-7 (FP32), 2.2e-7 (FP16S)
