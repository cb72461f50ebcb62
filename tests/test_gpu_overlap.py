"""Detection overlapped with the dynamics on one GPU (the active set updated
in the shadow of the dynamics, Sec. 2.2): the next active set is built on a
second stream from a snapshot of the state while the steps go on, and taken
into use one interval later, with margins covering two intervals.

With zero missed contacts the trajectory is the one per-step detection
gives, bit for bit: fixed rule and learned envelopes, the all-FP64 and the
FP32-force modes; a margin cap too small for the motion makes the guard
re-detect on the step's stream, still bit for bit; a storage too small for
the set built ahead is grown and the run stays bit-identical."""
import numpy as np
import pytest

from paper_2307_03445_amd import inputs as I

pytestmark = pytest.mark.gpu


def _scene(desc, prec="fp64"):
    from paper_2307_03445_amd._lib import Scene
    return Scene(desc, precision=prec)


@pytest.fixture(scope="module")
def dense():
    return I.walled_box(dense=True)


@pytest.fixture(scope="module")
def mlp():
    from paper_2307_03445_amd import train
    p = train.load_weights()
    assert p is not None
    return p


def _run(desc, prec, steps, mode=None, mlp=None, **det):
    sc = _scene(desc, prec)
    if mode == "learned":
        sc.set_mlp(mlp)
    if mode:
        sc.set_detection(mode, **det)
    sc.step(steps)
    out = sc.state(), sc.counts()
    sc.close()
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", ["fixed", "learned"])
def test_overlap_equals_per_step_detection(dense, mlp, prec, mode):
    steps = 160
    ref, _ = _run(dense, prec, steps)
    st, c = _run(dense, prec, steps, mode, mlp, k_max=10, safety=1.5, margin_cap=1e-4, audit_period=25,
                 overlap=True)
    print(mode, prec, c, flush=True)
    for k in ("x", "q", "v", "w"):
        assert np.array_equal(st[k], ref[k]), k
    assert c["missed"] == 0 and c["audits"] >= 6
    # one detection at the start, then one set adopted per interval
    assert steps // 10 - 1 <= c["detections"] <= steps // 10 + 2 + c["guard_trips"], c


def test_guard_redetects_when_margins_are_too_small(dense):
    """Margins capped far below the motion of two intervals: spheres outrun
    them, the guard re-detects on the step's stream, and the trajectory is
    still the per-step one."""
    steps = 120
    ref, _ = _run(dense, "fp64", steps)
    st, c = _run(dense, "fp64", steps, "fixed", k_max=10, safety=1.5, margin_cap=2e-7, audit_period=20,
                 overlap=True)
    print(c, flush=True)
    for k in ("x", "q", "v", "w"):
        assert np.array_equal(st[k], ref[k]), k
    assert c["guard_trips"] > 0 and c["missed"] == 0


def test_storage_grown_for_the_set_built_ahead(dense, monkeypatch):
    monkeypatch.setenv("CDEM_INITIAL_CAPACITY", "512")
    small = _scene(dense)
    monkeypatch.delenv("CDEM_INITIAL_CAPACITY")
    small.set_detection("fixed", k_max=10, safety=1.5, margin_cap=1e-4, audit_period=20, overlap=True)
    small.step(60)
    c = small.counts()
    ref, _ = _run(dense, "fp64", 60)
    st = small.state()
    small.close()
    assert c["regrows"] >= 1 and c["missed"] == 0, c
    for k in ("x", "q", "v", "w"):
        assert np.array_equal(st[k], ref[k]), k


def test_overlap_across_calls_and_switching_it_off(dense):
    """The pipeline carries over from one call to the next (a set in flight
    at the end of a call is adopted in the next), and switching the overlap
    off and on again keeps the trajectory."""
    ref, _ = _run(dense, "fp32", 100)
    sc = _scene(dense, "fp32")
    sc.set_detection("fixed", k_max=8, safety=1.5, margin_cap=1e-4, audit_period=0, overlap=True)
    for n in (3, 17, 9, 11):  # 40 steps in uneven calls
        sc.step(n)
    sc.set_detection("fixed", k_max=8, safety=1.5, margin_cap=1e-4, audit_period=0)
    sc.step(30)
    sc.set_detection("fixed", k_max=5, safety=1.5, margin_cap=1e-4, audit_period=0, overlap=True)
    sc.step(30)
    st = sc.state()
    sc.close()
    for k in ("x", "q", "v", "w"):
        assert np.array_equal(st[k], ref[k]), k
