"""Checkpoints (cdem_save / cdem_load): a scene saved after n steps and
restored into a fresh scene of the same description continues bit for bit as
the uninterrupted run, in every precision and detection mode; blobs of another
description or of the wrong size are refused."""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2307_03445_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dense():
    return I.walled_box(dense=True)


def _params():
    g = np.random.default_rng(11)
    p = M.init_params(g, mu=(-3.0, 3.0, 2.5), sig=(1.5, 2.0, 1.0)).astype(np.float32)
    p[M.OFF_B3:M.OFF_B3 + 2] = (-1.0, 4.0)
    return p


def _make(desc, prec, mode):
    from paper_2307_03445_amd._lib import Scene
    sc = Scene(desc, precision=prec)
    if mode == "learned":
        sc.set_mlp(_params())
    if mode != "plain":
        sc.set_detection(mode, k_max=20, safety=1.5, margin_cap=1e-4, audit_period=50)
    return sc


@pytest.mark.parametrize("prec,mode", [("fp64", "plain"), ("fp64", "fixed"), ("fp32", "fixed"), ("fp32", "learned")])
def test_save_load_resumes_bitwise(dense, prec, mode):
    a = _make(dense, prec, mode)
    a.step(97)  # mid-interval for the deferred modes
    blob = a.save()
    a.step(103)
    ref = a.state()
    b = _make(dense, "fp64" if prec == "fp32" else "fp32", "plain")
    with pytest.raises(Exception):
        b.load(blob)  # other precision: refused
    b = _make(dense, prec, "plain")  # settings come from the checkpoint
    b.load(blob)
    assert b.counts()["steps"] == 97
    b.step(103)
    got = b.state()
    for k in ref:
        assert np.array_equal(ref[k], got[k]), k
    assert b.counts()["missed"] == 0


def test_load_rejects_foreign_or_truncated_blob(dense):
    a = _make(dense, "fp64", "plain")
    a.step(5)
    blob = a.save()
    other = I.walled_box(replica=1, dense=True)  # same counts, other templates
    b = _make(other, "fp64", "plain")
    for bad in (blob[:-8], blob[:100], b"x" * len(blob)):
        with pytest.raises(Exception):
            a.load(bad)
    with pytest.raises(Exception):
        b.load(blob)
    a.load(blob)  # its own blob still loads after the refusals
    assert a.counts()["steps"] == 5
