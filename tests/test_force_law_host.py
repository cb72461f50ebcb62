"""User force laws compiled at run time (hiprtc, gfx950) without a device:
the laws the GPU tests use compile, and a broken law is refused with the
compiler's message pointing into the user's source."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def _law(name):
    with open(os.path.join(HERE, "laws", name)) as fh:
        return fh.read()


def test_the_test_laws_compile():
    from paper_2307_03445_amd import _lib
    for name in ("hertz_mindlin.hip", "linear_dashpot.hip"):
        ok, log = _lib.check_force_law(_law(name))
        assert ok, (name, log)


def test_a_broken_law_is_refused_with_the_compiler_message():
    from paper_2307_03445_amd import _lib
    src = _law("linear_dashpot.hip").replace("const double f = k * delta - c * vn;", "const double f = k * dlta;")
    ok, log = _lib.check_force_law(src)
    assert not ok
    assert "user_law:" in log and "dlta" in log, log


def test_a_law_with_the_wrong_signature_is_refused():
    from paper_2307_03445_amd import _lib
    ok, log = _lib.check_force_law("__device__ void cdem_user_law(double *F) { F[0] = 0.0; }")
    assert not ok and "cdem_user_law" in log, log
