"""Deferred active-set updates (paper Sec. 2.2): detection every k steps with
enlarged contact geometry must reproduce per-step detection exactly, because
false-positive candidates exert no force and the reduction order is fixed."""
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


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fixed_rule_bitwise_equals_plain(dense, prec):
    plain, fixed = _scene(dense, prec), _scene(dense, prec)
    fixed.set_detection("fixed", k_max=20, safety=1.5, margin_cap=1e-4, audit_period=10)
    plain.step(200)
    fixed.step(200)
    sp, sf = plain.state(), fixed.state()
    for k in sp:
        assert np.array_equal(sp[k], sf[k]), k
    c = fixed.counts()
    assert c["detections"] < 100, c          # detection really was deferred
    assert c["audits"] >= 19 and c["missed"] == 0, c
    assert c["candidates"] >= plain.counts()["candidates"]


def test_guard_forces_early_redetection():
    """Clumps released at rest with overlaps: the first detection sees zero
    speed, so only the displacement guard keeps the active set complete."""
    d = I.walled_box(dense=True, vel_noise=0.0)
    plain, fixed = _scene(d), _scene(d)
    fixed.set_detection("fixed", k_max=20, safety=1.0, margin_cap=1e-4, audit_period=5)
    plain.step(100)
    fixed.step(100)
    c = fixed.counts()
    assert c["guard_trips"] >= 1 and c["missed"] == 0, c
    sp, sf = plain.state(), fixed.state()
    for k in sp:
        assert np.array_equal(sp[k], sf[k]), k


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_guard_bound_keeps_the_per_sphere_trip_schedule(prec, monkeypatch):
    """The guard skips the per-sphere test for clumps whose CoM displacement
    plus rotation bound stays below their smallest margin; a testing switch
    turns the bound off, and the guard must trip on exactly the same steps."""
    d = I.walled_box(dense=True, vel_noise=0.0)
    monkeypatch.setenv("CDEM_TEST_EXACT_GUARD", "1")
    ref = _scene(d, prec)
    monkeypatch.delenv("CDEM_TEST_EXACT_GUARD")
    fast = _scene(d, prec)
    for sc in (ref, fast):
        sc.set_detection("fixed", k_max=20, safety=1.0, margin_cap=1e-4, audit_period=5)
    for step in range(150):
        ref.step(1)
        fast.step(1)
        cr, cf = ref.counts(), fast.counts()
        assert (cr["guard_trips"], cr["detections"]) == (cf["guard_trips"], cf["detections"]), (step, cr, cf)
    assert cf["guard_trips"] >= 1 and cf["missed"] == 0, cf
    sr, sf = ref.state(), fast.state()
    for k in sr:
        assert np.array_equal(sr[k], sf[k]), k


def test_audit_reports_misses_when_guard_disabled(dense, monkeypatch):
    """Failure path forced from the host: a testing switch removes the margin
    and the guard (detection every 20 steps with the exact predicate), so
    contacts that form between detections are missing and the periodic audit
    must report them."""
    from paper_2307_03445_amd._lib import CdemError
    monkeypatch.setenv("CDEM_TEST_NO_GUARD", "1")
    sc = _scene(dense)
    monkeypatch.delenv("CDEM_TEST_NO_GUARD")
    sc.set_detection("fixed", k_max=20, safety=1.0, margin_cap=1e-4, audit_period=3)
    with pytest.raises(CdemError) as e:
        sc.step(200)
    assert e.value.code == -5
    assert sc.counts()["missed"] > 0


def test_write_state_keeps_history_and_redetects(dense):
    """Writing the state back unchanged forces a rebuild that keeps every
    surviving pair's history, so the trajectory is unchanged."""
    a, b = _scene(dense), _scene(dense)
    a.step(30)
    b.step(30)
    b.write_state(**b.state())
    a.step(30)
    b.step(30)
    sa, sb = a.state(), b.state()
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k


def test_invalid_detection_parameters_rejected(dense):
    from paper_2307_03445_amd._lib import CdemError
    sc = _scene(dense)
    for kw in (dict(k_max=0), dict(k_max=21), dict(safety=0.5), dict(margin_cap=0.0)):
        args = dict(mode="fixed", k_max=5, safety=1.5, margin_cap=1e-4)
        args.update(kw)
        with pytest.raises(CdemError):
            sc.set_detection(**args)


@pytest.mark.parametrize("mode", ["fixed", "learned"])
def test_regrow_on_an_audit_step_reports_no_miss(dense, mode, monkeypatch):
    """An active set too small for the first detection overflows on a step
    that also audits (step 0, audit period 10).  The abandoned step must not
    be audited; it is run again once the storage has grown, so the call
    succeeds, the audits count no miss, and the trajectory is bit-identical
    to a scene that never had to grow."""
    from paper_2307_03445_amd import train
    mlp = np.load(train.WEIGHTS)["params"].astype(np.float32) if mode == "learned" else None

    def make():
        sc = _scene(dense)
        if mlp is not None:
            sc.set_mlp(mlp)
        sc.set_detection(mode, k_max=20, safety=1.5, margin_cap=1e-4, audit_period=10)
        return sc

    monkeypatch.setenv("CDEM_INITIAL_CAPACITY", "512")
    small = make()
    monkeypatch.delenv("CDEM_INITIAL_CAPACITY")
    ref = make()
    small.step(30)  # raises CdemError on a reported miss
    ref.step(30)
    c = small.counts()
    assert c["regrows"] >= 1 and c["audits"] == 3 and c["missed"] == 0, c
    assert ref.counts()["missed"] == 0
    s1, s2 = small.state(), ref.state()
    for k in s1:
        assert np.array_equal(s1[k], s2[k]), k
