"""Host logic of the PyTorch binding that needs no GPU: plans and batches
released while the current stream is being captured are queued and destroyed,
in release order, at the first release or creation outside the capture."""
import pytest

from paper_2604_07248_amd import api


@pytest.fixture
def capture(monkeypatch):
    state = {"on": False}
    monkeypatch.setattr(api, "_capturing", lambda: state["on"])
    monkeypatch.setattr(api, "_deferred", [])
    return state


def test_release_outside_capture_is_immediate(capture):
    done = []
    api._release(done.append, "h1")
    assert done == ["h1"] and api._deferred == []


def test_release_inside_capture_is_deferred_then_flushed_in_order(capture):
    done = []
    capture["on"] = True
    api._release(done.append, "h1")
    api._release(done.append, "h2")
    api._flush_deferred()  # still capturing: nothing happens
    assert done == [] and [h for _, h in api._deferred] == ["h1", "h2"]
    capture["on"] = False
    api._release(done.append, "h3")  # the queue goes first
    assert done == ["h1", "h2", "h3"] and api._deferred == []


def test_flush_outside_capture(capture):
    done = []
    capture["on"] = True
    api._release(done.append, "h1")
    capture["on"] = False
    api._flush_deferred()
    assert done == ["h1"] and api._deferred == []
