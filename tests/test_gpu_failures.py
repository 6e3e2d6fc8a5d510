"""Failure handling of the solver context (include/qs.h, qs_sync_check): a non-finite state
or a stalled xi-segment hand-off is reported with its instance, mode and step; with the
rollback copy enabled the state is restored to the last good tau-step, otherwise the context
refuses to step until its state is replaced.  The failures are forced from the host: an
FP32 state stored next to the top of the float range overflows in the next sweep, and a
zero wait budget makes every hand-off wait give up (each wave still exits)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _inst(**kw):
    """Slab beam with a long step (Gamma_CFI d_tau ~ 0.6 at the largest k: a sweep of two
    steps multiplies the fastest modes by ~3)."""
    from paper_2607_24234_amd import inputs
    d = inputs.slab(n_modes=6, n_xi=96, n_steps=4)
    d["d_tau"] = 200.0
    d.update(kw)
    return d


def _near_overflow(st, mode):
    """The state with mode `mode` (a growing one) scaled so that its largest stored FP32 value
    is 0.999 of the float range: finite as stored, past the range after the next sweep."""
    out = [{k: v.copy() for k, v in s.items()} for s in st]
    s = out[0]
    mx = max(np.max(np.abs(s[key][mode].view(np.float64))) for key in ("rho", "j_par", "j_perp"))
    f = 0.999 * float(np.finfo(np.float32).max) / mx
    for key in ("rho", "j_par", "j_perp"):
        s[key][mode] *= f
    s["log2_scale"][mode] = 0.0
    return out


def _physical(st):
    s = st[0]
    f = 2.0 ** s["log2_scale"][:, None]
    return s["rho"] * f, s["j_par"] * f, s["j_perp"] * f


def test_nonfinite_rolls_back_to_last_good_step(qs):
    s = qs.Solver([_inst()], precision=qs.QS_FP32)
    s.set_rollback(True)
    s.step(3)
    s.sync_check()
    bad = _near_overflow(s.get_state(), 5)
    s.set_state(bad)
    before = s.get_state()
    s.step(2)
    with pytest.raises(qs.QSError) as e:
        s.sync_check()
    assert e.value.status == qs.QS_ERR_NUMERIC
    msg = str(e.value)
    assert "instance 0, mode 5" in msg and "after tau-step" in msg and "rolled back to tau-step 3" in msg
    assert s.steps_done == 3
    after = s.get_state()
    for a, b in zip(_physical(before), _physical(after)):
        assert np.array_equal(a, b)
    # the context goes on: a normal state steps and checks clean, and the step count goes on
    s.set_state(qs.Solver([_inst()], precision=qs.QS_FP32).get_state())
    s.step(2)
    s.sync_check()
    assert s.steps_done == 5


def test_nonfinite_without_rollback_poisons_the_context(qs):
    s = qs.Solver([_inst()], precision=qs.QS_FP32)
    s.step(2)
    s.set_state(_near_overflow(s.get_state(), 5))
    s.step(3)
    with pytest.raises(qs.QSError) as e:
        s.sync_check()
    # steps 3 and 4 share one sweep, after which the stored state is checked
    assert e.value.status == qs.QS_ERR_NUMERIC and "mode 5" in str(e.value) and "after tau-step 4" in str(e.value)
    with pytest.raises(qs.QSError) as e:
        s.step(1)
    assert e.value.status == qs.QS_ERR_STATE
    s.sync_check()                      # reported once
    s.set_state(qs.Solver([_inst()], precision=qs.QS_FP32).get_state())
    s.step(1)
    s.sync_check()


def test_step_numbers_count_graph_replays(qs):
    """The reported step comes from the device's own step counter, which graph replays
    advance like eager calls."""
    inst = _inst()
    s = qs.Solver([inst], precision=qs.QS_FP32)
    g = qs.Graph(s, 2)
    g.replay()
    g.replay()
    s.sync_check()
    assert s.steps_done == 4
    s.set_state(_near_overflow(s.get_state(), 5))
    g.replay()
    with pytest.raises(qs.QSError) as e:
        s.sync_check()
    assert "mode 5" in str(e.value) and "after tau-step 6" in str(e.value)
    with pytest.raises(qs.QSError) as e:
        g.replay()
    assert e.value.status == qs.QS_ERR_STATE
    g.close()


@pytest.mark.parametrize("rollback", [False, True])
def test_stalled_handoff_reported(qs, rollback):
    """Eight xi-segments per block with a zero wait budget: the hand-off waits give up, every
    wave exits, and qs_sync_check reports the stall; with the rollback copy the state of the
    start of the call comes back bitwise."""
    inst = _inst(n_xi=296)
    s = qs.Solver([inst], precision=qs.QS_FP32, segment_cells=37)
    assert s.plan()["max_segments"] == 8
    if rollback:
        s.set_rollback(True)
    s.step(2)
    s.sync_check()
    before = s.get_state()
    s.debug_wait_budget(0.0)
    s.step(4)
    with pytest.raises(qs.QSError) as e:
        s.sync_check()
    assert e.value.status == qs.QS_ERR_HIP and "hand-off wait gave up" in str(e.value)
    s.debug_wait_budget(-1.0)
    if rollback:
        assert s.steps_done == 2
        for a, b in zip(_physical(before), _physical(s.get_state())):
            assert np.array_equal(a, b)
        s.step(1)
        s.sync_check()
    else:
        with pytest.raises(qs.QSError) as e:
            s.step(1)
        assert e.value.status == qs.QS_ERR_STATE
