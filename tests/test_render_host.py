"""Host logic of the batched render proxy, on the CPU: the query-packet
context sets the tree's query packet for the shadow and hit-point queries
and always restores it, also when the query fails."""
import types

import pytest

from paper_2405_16788_amd import binding as B
from workloads import render as R


@pytest.fixture
def launch(monkeypatch):
    state = {"query": 4, "adjoint": 2, "flags": 12}
    calls = []

    def get(tree):
        return dict(state)

    def set_(tree, q, a, f):
        calls.append((q, a, f))
        if q:
            state["query"] = q
        if a:
            state["adjoint"] = a
        if f >= 0:
            state["flags"] = f

    monkeypatch.setattr(B, "dps_get_launch", get)
    monkeypatch.setattr(B, "dps_set_launch", set_)
    return state, calls


def test_packet_set_and_restored(launch):
    state, calls = launch
    tree = types.SimpleNamespace()
    with R._query_packet(tree, 1):
        assert state == {"query": 1, "adjoint": 2, "flags": 12}
    assert state == {"query": 4, "adjoint": 2, "flags": 12}
    assert calls == [(1, 0, -1), (4, 0, -1)]


def test_packet_restored_on_error(launch):
    state, _ = launch
    with pytest.raises(RuntimeError):
        with R._query_packet(types.SimpleNamespace(), 2):
            raise RuntimeError("query failed")
    assert state["query"] == 4


def test_none_leaves_the_tree_alone(launch):
    state, calls = launch
    with R._query_packet(types.SimpleNamespace(), None):
        pass
    assert calls == [] and state["query"] == 4
