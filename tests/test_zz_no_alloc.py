"""yy_step_static -- the step of yy_step with its scratch arrays in the
library's static device array, for callers that cannot allocate -- checked
against yy_step itself through the C-ABI: two calls in a row on the same
GPU, the second on a smaller grid (the static array keeps the first call's
contents), FP64 and FP32-mixed, with the mass-flux correction and the
pressure exchange on in the first (they use the partial sums and the
Thomas scratch); and a grid whose scratch does not fit is refused."""
import numpy as np
import pytest

from paper_1905_02300_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def yy():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1905_02300_amd import yy as mod
    mod.load()
    return mod


def _convection_pair(yy, nr, nt, np_, prec, ra, seed):
    grid = I.Grid(nr, nt, np_)
    st = I.convection_state(grid, 1.0, ra, seed=seed)
    shells = []
    for _ in range(2):
        sh = yy.Shell(nr, nt, np_, prec=prec)
        sh.set_params(pr=1.0, ra=ra, dt=2e-4, t_inner=1.0)
        for f in range(9):
            sh.set_field(f, 0, st[f])
            if f not in (I.P1, I.P2):
                sh.set_field(f, 1, st[f])
        shells.append(sh)
    return shells


def _same(a, b, K, prec):
    for f in range(9):
        x = a.get_field(f).cpu().numpy()
        y = b.get_field(f).cpu().numpy()
        if prec == 0:
            scale = max(np.max(np.abs(y)), 1e-300)
            assert np.max(np.abs(x - y)) <= 1e-12 * scale, I.FIELD_NAMES[f]
        else:
            assert np.array_equal(x, y), I.FIELD_NAMES[f]
    assert np.array_equal(a.norms(), b.norms())


@pytest.mark.parametrize("prec", [0, 1])
def test_step_static_matches_step(yy, prec):
    # first call: 12x30x90 with the mass-flux correction and the pressure
    # exchange on (they use the partial sums and the Thomas scratch)
    print(f"case: static step, prec {prec}, 12x30x90 then 6x12x36", flush=True)
    a, b = _convection_pair(yy, 12, 30, 90, prec, 1e5, 3)
    for sh in (a, b):
        sh.set_mass_fix(True)
        sh.set_pressure_exchange(1)
    for _ in range(2):
        a.step(3)
        b.step_static(3)
    _same(a, b, 3, prec)
    # second call, a smaller grid on the same static array, with the
    # LDS-staged residual tiles
    a, b = _convection_pair(yy, 6, 12, 36, prec, 1e4, 4)
    for sh in (a, b):
        sh.set_tuning('{"res.T":"lds64x4k","res.u_r":"lds64x8k","res.u_t":"lds64x4k","res.u_p":"lds64x8j"}')
    for _ in range(3):
        a.step(2)
        b.step_static(2)
    _same(a, b, 2, prec)


def test_step_static_refuses_oversize_grid(yy):
    """A grid whose residual buffer exceeds the static array's 32 MiB per
    array is refused before any device work."""
    print("case: static step refuses 48x128x384", flush=True)
    sh = yy.Shell(48, 128, 384)
    sh.set_params(pr=1.0, ra=0.0, dt=1e-3)
    with pytest.raises(yy.YYError) as e:
        sh.step_static(1)
    assert e.value.status == yy.YY_ERR_WORKSPACE
