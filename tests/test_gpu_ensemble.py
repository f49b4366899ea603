"""Ensembles of independent shells (uneven sizes and Rayleigh numbers)
advanced by the captured graphs: each shell against its own oracle shell,
the FP32-mixed ensemble against graph-free stepping and against FP64,
single-shell steps interleaved with graph steps, and the refusal of shells
with wall data."""
import numpy as np
import pytest

from paper_1905_02300_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GRIDS = [(6, 12, 36), (10, 20, 60), (8, 16, 48)]
RAS = [1e3, 1e4, 1e5]
DT, K = 2e-4, 3


@pytest.fixture(scope="module")
def yy():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1905_02300_amd import yy as mod
    mod.load()
    return mod


def _states(grids=GRIDS, ras=RAS):
    return [I.convection_state(I.Grid(*g), 1.0, ra, seed=1000 + q) for q, (g, ra) in enumerate(zip(grids, ras))]


def _load_ensemble(yy, prec, states, grids=GRIDS, ras=RAS):
    e = yy.Ensemble(grids, prec=prec)
    for q, sh in enumerate(e.shells):
        sh.set_params(pr=1.0, ra=ras[q], dt=DT, t_inner=1.0)
        for f in range(9):
            sh.set_field(f, 0, states[q][f])
            if f not in (I.P1, I.P2):
                sh.set_field(f, 1, states[q][f])
    return e


def test_ensemble_graph_matches_oracle(oracle_lib, yy):
    """Three FP64 shells stepped by graph replay over more than one cycle
    of the six level-rotation phases (8 steps), each compared with its own
    oracle shell: 1e-12 relative, the velocities plus the rounding floor of
    the cancelling buoyancy and hydrostatic pressure gradient."""
    print("case: FP64 ensemble graph vs oracle", flush=True)
    states = _states()
    e = _load_ensemble(yy, yy.YY_FP64, states)
    nsteps = 8
    for _ in range(nsteps):
        e.step(K, graph=True)
    for q, (g, ra) in enumerate(zip(GRIDS, RAS)):
        o = oracle_lib.Shell(*g)
        o.set_params(pr=1.0, ra=ra, tau=DT, chi=1.0, t_inner=1.0, t_outer=0.0)
        for f in range(9):
            o.set_field(f, 0, states[q][f])
            if f not in (I.P1, I.P2):
                o.set_field(f, 1, states[q][f])
        for _ in range(nsteps):
            o.step(K)
        floor = 16 * np.finfo(float).eps * DT * ra * np.max(np.abs(states[q][I.T])) * nsteps * K
        for f in range(9):
            a = e.shells[q].get_field(f).cpu().numpy()
            b = o.get_field(f)
            err = np.max(np.abs(a - b))
            lim = 1e-12 * np.max(np.abs(b)) + (0.0 if f in (I.T, I.P1, I.P2) else floor)
            assert err <= lim, (q, I.FIELD_NAMES[f], err, lim)


def test_ensemble_fp32_graph_autotuned(yy):
    """FP32-mixed ensemble with each shell's tiles from the autotuner: the
    graph replay equals graph-free stepping bitwise, and the result stays
    within the FP32-mixed error of the FP64 ensemble (T stored as its
    deviation from the conductive profile: T and p at 1e-7 relative, the
    velocity, a small response to 1e-3 temperature noise under a 1e5
    hydrostatic balance, at 1e-5 relative; measured 2e-9, 2e-10, 3e-7)."""
    print("case: FP32 ensemble graph vs eager vs FP64", flush=True)
    states = _states()
    ens = [_load_ensemble(yy, yy.YY_FP32_MIXED, states) for _ in range(2)]
    js = [sh.autotune() for sh in ens[0].shells]
    for sh, j in zip(ens[1].shells, js):
        sh.set_tuning(j)
    ref = _load_ensemble(yy, yy.YY_FP64, states)
    for _ in range(8):
        ens[0].step(K, graph=True)
        ens[1].step(K, graph=False)
        ref.step(K, graph=True)
    for q in range(len(GRIDS)):
        for f in range(9):
            a = ens[0].shells[q].get_field(f).cpu().numpy()
            b = ens[1].shells[q].get_field(f).cpu().numpy()
            assert np.array_equal(a, b), (q, I.FIELD_NAMES[f])
            c = ref.shells[q].get_field(f).cpu().numpy()
            rel = np.max(np.abs(a - c)) / np.max(np.abs(c))
            lim = 1e-7 if f in (I.T, I.P1, I.P2) else 1e-5
            print(f"  shell {q} {I.FIELD_NAMES[f]}: FP32-mixed vs FP64 {rel:.2e}")
            assert rel <= lim, (q, I.FIELD_NAMES[f], rel)


@pytest.mark.parametrize("prec", [0, 1])
def test_ensemble_batched_equals_streams_and_eager(yy, prec):
    """The batched graph (per branch of shells, one launch per step position
    and tile bin, each shell owning a range of blocks) with per-bucket tiles
    from the ensemble
    autotuner gives bitwise the results of the per-shell stream graph and
    of graph-free stepping, over more than one rotation cycle; and it is
    batched: fewer launches per step than the shells' launches together."""
    print(f"case: ensemble batched vs streams vs eager, prec {prec}", flush=True)
    # eight shells, so that the four branches batch two shells each
    grids = GRIDS + [(6, 14, 42), (12, 12, 36), (6, 12, 36), (10, 22, 66), (8, 18, 54)]
    ras = RAS + [3e3, 3e4, 1e3, 1e5, 1e4]
    states = _states(grids, ras)
    ens = [_load_ensemble(yy, prec, states, grids, ras) for _ in range(3)]
    tiles = ens[0].autotune()
    assert "n<=" in tiles
    # the same tiles on every copy (the tuner's timings may pick others)
    for e in ens[1:]:
        for sh, src in zip(e.shells, ens[0].shells):
            sh.set_tuning(src.tuning_json())
    for _ in range(8):
        ens[0].step(K, graph=1)
        ens[1].step(K, graph=2)
        ens[2].step(K, graph=0)
    batched, launches, own = ens[0].info()
    print(f"  batched launches per step {launches}, the shells' own {own}", flush=True)
    assert batched and 0 < launches < own
    for q in range(len(grids)):
        for f in range(9):
            a = ens[0].shells[q].get_field(f).cpu().numpy()
            b = ens[1].shells[q].get_field(f).cpu().numpy()
            c = ens[2].shells[q].get_field(f).cpu().numpy()
            assert np.array_equal(a, b) and np.array_equal(a, c), (q, I.FIELD_NAMES[f])
        assert np.array_equal(ens[0].shells[q].norms(), ens[2].shells[q].norms())


def test_ensemble_member_steps_between_graph_steps(yy):
    """A single-shell step on one member between graph steps (the level
    pointers then rotate outside the captured graphs): the graphs are
    captured again, and every shell ends bitwise equal to the same sequence
    stepped without graphs."""
    print("case: ensemble with interleaved single-shell steps", flush=True)
    states = _states()
    a = _load_ensemble(yy, yy.YY_FP64, states)
    b = _load_ensemble(yy, yy.YY_FP64, states)
    for n in range(7):
        a.step(K, graph=True)
        b.step(K, graph=False)
        if n in (1, 4):
            a.shells[1].step(K)
            b.shells[1].step(K)
        if n == 2:
            a.shells[2].step_tol(5, 1e-30)
            b.shells[2].step_tol(5, 1e-30)
    for q in range(len(GRIDS)):
        for f in range(9):
            x = a.shells[q].get_field(f).cpu().numpy()
            y = b.shells[q].get_field(f).cpu().numpy()
            assert np.array_equal(x, y), (q, I.FIELD_NAMES[f])


def test_ensemble_graph_refuses_wall_data(yy):
    """A shell with wall data cannot be replayed (its wall values change
    every step): the graph step is refused before anything advances, and
    graph-free stepping still works."""
    print("case: ensemble refuses wall data under graph", flush=True)
    states = _states()
    a = _load_ensemble(yy, yy.YY_FP64, states)
    b = _load_ensemble(yy, yy.YY_FP64, states)
    for e in (a, b):
        g = I.Grid(*GRIDS[0])
        w = np.zeros((2, g.nt + 2, g.np + 2))
        for lev in (0, 1, 2):
            e.shells[0].set_wall(I.T, lev, 0, w + 1.0)
    with pytest.raises(yy.YYError) as err:
        a.step(K, graph=True)
    assert err.value.status == yy.YY_ERR_STATE
    for e in (a, b):
        g = I.Grid(*GRIDS[0])
        e.shells[0].set_wall(I.T, 2, 0, np.ones((2, g.nt + 2, g.np + 2)))
        e.step(K, graph=False)
    for q in range(len(GRIDS)):
        for f in range(9):
            x = a.shells[q].get_field(f).cpu().numpy()
            y = b.shells[q].get_field(f).cpu().numpy()
            assert np.array_equal(x, y), (q, I.FIELD_NAMES[f])


def test_ensemble_batched_falls_back_for_mass_fix_and_exchange(yy):
    """The mass fix and the pressure exchange have no batched kernels: an
    ensemble with such a shell is captured as per-shell streams instead
    (info reports not batched), and stays bitwise equal to graph-free
    stepping; without them it is batched again."""
    print("case: ensemble batched fallback (mass fix, pressure exchange)", flush=True)
    states = _states()
    a = _load_ensemble(yy, yy.YY_FP64, states)
    b = _load_ensemble(yy, yy.YY_FP64, states)
    for e in (a, b):
        e.shells[0].set_mass_fix(1)
        e.shells[2].set_pressure_exchange(1)
    for _ in range(3):
        a.step(K, graph=1)
        b.step(K, graph=0)
    assert a.info()[0] is False
    for e in (a, b):
        e.shells[0].set_mass_fix(0)
        e.shells[2].set_pressure_exchange(0)
    for _ in range(3):
        a.step(K, graph=1)
        b.step(K, graph=0)
    assert a.info()[0] is True
    for q in range(len(GRIDS)):
        for f in range(9):
            x = a.shells[q].get_field(f).cpu().numpy()
            y = b.shells[q].get_field(f).cpu().numpy()
            assert np.array_equal(x, y), (q, I.FIELD_NAMES[f])


def test_ensemble_batched_multiplicative_and_mixed_modes(yy):
    """Shells in the multiplicative mode (Yin, then Yang from Yin's
    iterate: one patch per launch) batch like additive ones and stay
    bitwise equal to graph-free stepping; an ensemble mixing the two modes
    has step sequences that do not line up, so it takes the per-shell
    stream graph (info: not batched) with the same results."""
    print("case: ensemble batched, multiplicative and mixed modes", flush=True)
    states = _states()
    for modes, want_batched in (([1, 1, 1], True), ([0, 1, 0], False)):
        a = _load_ensemble(yy, yy.YY_FP64, states)
        b = _load_ensemble(yy, yy.YY_FP64, states)
        for e in (a, b):
            for q, sh in enumerate(e.shells):
                sh.set_params(pr=1.0, ra=RAS[q], dt=DT, t_inner=1.0, mode=modes[q])
        for _ in range(7):
            a.step(K, graph=1)
            b.step(K, graph=0)
        assert a.info()[0] is want_batched, modes
        for q in range(len(GRIDS)):
            for f in range(9):
                x = a.shells[q].get_field(f).cpu().numpy()
                y = b.shells[q].get_field(f).cpu().numpy()
                assert np.array_equal(x, y), (modes, q, I.FIELD_NAMES[f])
