"""Helpers for GPU tests: device transfers and model construction (no solver arithmetic)."""
import sys

import numpy as np
import pytest

from rte_inputs import configs, weights


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(a, dtype="float64"):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", getattr(torch, dtype))


def host(t):
    return t.detach().cpu().numpy()


def model_for(prob):
    from paper_2604_23265_amd import api
    hdr, t = configs.problem_weights(prob)
    blob = weights.pack_mgn1(hdr, t)
    return api.Model(blob), blob


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
