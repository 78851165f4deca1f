"""Host logic of the autograd wrapper, on the CPU with the library calls
replaced by recorders: the forward asks the native query for spatial
gradients exactly when the caller wants them (a values-only call must not
pay for the gradient kernel), on the full and the channel-subset paths."""
import types

import pytest
import torch

from paper_2405_16788_amd import autograd as AG


class _Recorder:
    def __init__(self):
        self.calls = []

    def query(self, tree, x, beta, eps, grad=True, f_out=None, g_out=None):
        self.calls.append(("query", grad, g_out))
        Q = x.shape[0]
        return torch.zeros((Q, tree.C)), (torch.zeros((Q, tree.C, 3)) if grad else None)

    def query_channels(self, tree, x, beta, eps, c_begin, n, grad=True, f_out=None, g_out=None, q_count=None):
        self.calls.append(("channels", grad, g_out))
        return f_out, g_out


@pytest.fixture
def rec(monkeypatch):
    r = _Recorder()
    monkeypatch.setattr(AG.B, "dps_query", r.query)
    monkeypatch.setattr(AG.B, "dps_query_channels", r.query_channels)
    monkeypatch.setattr(AG, "_refit", lambda tree, attrs, mode: None)
    return r


def _tree(C=4):
    return types.SimpleNamespace(C=C, kernel="dipole")


@pytest.mark.parametrize("grad", [False, True])
def test_channel_subset_forwards_the_gradient_request(rec, grad):
    attrs, x = torch.zeros((10, 4)), torch.zeros((7, 3))
    f, g = AG.dipole_sum(attrs, x, _tree(), 2.0, 0.01, channels=(0, 1), grad=grad)
    kind, asked, g_out = rec.calls[-1]
    assert kind == "channels" and asked is grad
    assert (g_out is not None) is grad and (g is not None) is grad
    assert f.shape == (7, 1)


@pytest.mark.parametrize("grad", [False, True])
def test_row_count_path_forwards_the_gradient_request(rec, grad):
    attrs, x = torch.zeros((10, 4)), torch.zeros((7, 3))
    AG.dipole_sum(attrs, x, _tree(), 2.0, 0.01, q_count=torch.tensor([5]), grad=grad)
    kind, asked, _ = rec.calls[-1]
    assert kind == "channels" and asked is grad


@pytest.mark.parametrize("grad", [False, True])
def test_full_query_forwards_the_gradient_request(rec, grad):
    attrs, x = torch.zeros((10, 4)), torch.zeros((7, 3))
    f, g = AG.dipole_sum(attrs, x, _tree(), 2.0, 0.01, grad=grad)
    kind, asked, _ = rec.calls[-1]
    assert kind == "query" and asked is grad and (g is not None) is grad
