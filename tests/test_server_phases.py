"""Host logic of the server's training phases (no GPU): a generator's work
runs one phase per step, up to each yield and then to its end, and the
phase that finishes it says so; a plain callable counts as one phase that
ran when it was called."""
import pytest

pytest.importorskip("torch")

from paper_2409_04751_amd import server as S  # noqa: E402


def test_generator_runs_one_phase_per_step():
    log = []

    def view():
        log.append("forward")
        yield
        log.append("backward")

    ph = S._phases(view())
    assert next(ph) is False
    assert log == ["forward"]
    assert next(ph) is True  # the phase that finishes the view
    assert log == ["forward", "backward"]
    with pytest.raises(StopIteration):
        next(ph)


def test_plain_callable_is_one_phase():
    log = []
    ph = S._phases(log.append("step"))
    assert log == ["step"]
    assert next(ph) is True
    with pytest.raises(StopIteration):
        next(ph)


def test_run_phases_drains_generators():
    log = []

    def opt():
        for k in range(3):
            log.append(k)
            yield

    S.run_phases(opt())
    assert log == [0, 1, 2]
