"""Host-side lifetime rules of the batched plan binding (no GPU needed).

A captured graph holds kernels and stream dependencies recorded against the
plan's auxiliary streams, events and device tables, so it must be released
before the plan is destroyed (object teardown) or rebuilt (configuration
change). Releasing it afterwards left the runtime destroying a graph whose
capture resources were already gone.
"""
import ctypes

import pytest

from paper_1707_02018_amd import batched


class _FakeLib:
    def __init__(self, obj):
        self.obj = obj
        self.calls = []

    def aw_batch_destroy(self, plan):
        self.calls.append(("destroy", self.obj._graph is None, self.obj._graph_stream is None))
        return 0

    def aw_batch_set_config(self, plan, arr):
        self.calls.append(("set_config", self.obj._graph is None, self.obj._graph_stream is None))
        return 0


def _bare_plan():
    bf = object.__new__(batched.BatchedFista)
    bf._plan = ctypes.c_void_p(1)
    bf._graph = object()
    bf._graph_stream = object()
    bf.device = None
    return bf


def test_teardown_releases_graph_before_plan(monkeypatch):
    bf = _bare_plan()
    fake = _FakeLib(bf)
    monkeypatch.setattr(batched, "load", lambda: fake)
    bf.__del__()
    assert fake.calls == [("destroy", True, True)]
    assert bf._plan is None


def test_set_config_releases_graph_before_rebuild(monkeypatch):
    bf = _bare_plan()
    fake = _FakeLib(bf)
    monkeypatch.setattr(batched, "load", lambda: fake)
    monkeypatch.setattr(batched.torch.cuda, "synchronize", lambda *a, **k: None)
    bf.set_config((0, 1, 0, 2))
    assert fake.calls == [("set_config", True, True)]
    assert bf.config == (0, 1, 0, 2)
    bf._plan = None  # nothing to destroy at teardown
