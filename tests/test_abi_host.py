"""The C ABI on the host: exports, MGN1 parsing, input validation (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import problems
from rte_inputs import configs, weights

L = pytest.importorskip("paper_2604_23265_amd._lib")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("librte.so not built")
    return L.lib()


def test_every_declared_function_is_exported():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "rte.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"^\s*(?:rte_status|const char\*)\s+(\w+)\s*\(", hdr, flags=re.M))
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert names == set(L.exported_symbols())


def _load(blob):
    h = C.c_void_p()
    buf = C.create_string_buffer(blob, len(blob))
    return _lib().mgnet_load(buf, len(blob), C.byref(h)), h


def _blob(**mg):
    base = dict(c0=16, levels=3, nu_pre=2, nu_post=1, nu_coarse=2, coef_ch=3, seed=5)
    base.update(mg)
    hdr, t = weights.seeded_weights(2, 16, **base)
    return hdr, t


def test_mgnet_load_and_describe():
    hdr, t = _blob()
    code, h = _load(weights.pack_mgn1(hdr, t))
    assert code == 0
    d = (C.c_int * 8)()
    assert _lib().mgnet_describe(h, d) == 0
    assert list(d) == [2, 16, 16, 3, 2, 1, 2, 3]
    assert _lib().mgnet_free(h) == 0


def test_mgnet_load_accepts_any_tensor_order():
    hdr, t = _blob()
    keys = list(t)[::-1]
    code, h = _load(weights.pack_mgn1(hdr, t, order=keys))
    assert code == 0
    _lib().mgnet_free(h)


@pytest.mark.parametrize("mutate", ["magic", "truncate", "trailing", "missing", "shape", "dup", "version",
                                    "nan"])
def test_mgnet_load_rejects_corrupt_blobs(mutate):
    hdr, t = _blob()
    blob = weights.pack_mgn1(hdr, t)
    if mutate == "magic":
        blob = b"MGNX" + blob[4:]
    elif mutate == "truncate":
        blob = blob[: len(blob) // 2]
    elif mutate == "trailing":
        blob = blob + b"\x00" * 4
    elif mutate == "missing":
        t.pop(weights.tag(weights.K_R, 1))
        blob = weights.pack_mgn1(hdr, t)
    elif mutate == "shape":
        t[weights.tag(weights.K_A, 0)] = t[weights.tag(weights.K_A, 0)][:, :8]
        blob = weights.pack_mgn1(hdr, t)
    elif mutate == "dup":
        k = weights.tag(weights.K_S)
        blob = weights.pack_mgn1(dict(hdr), t, order=list(t) + [k])
    elif mutate == "version":
        blob = blob[:4] + (2).to_bytes(4, "little") + blob[8:]
    elif mutate == "nan":
        t[weights.tag(weights.K_A, 0)][0, 0, 0, 0] = np.nan
        blob = weights.pack_mgn1(hdr, t)
    code, h = _load(blob)
    assert code == L.RTE_EFORMAT
    assert _lib().rte_last_error().decode()


def test_mgnet_load_rejects_unsupported_channel_count():
    hdr, t = weights.seeded_weights(2, 8, 8, 2, seed=1)
    code, _ = _load(weights.pack_mgn1(hdr, t))
    assert code == L.RTE_EINVAL


def _build(prob, model=None):
    from paper_2604_23265_amd import api
    try:
        api.Operator(prob, model=model)
    except L.RteError as e:
        return e.code
    return 0


@pytest.mark.parametrize("bad", ["nan_sigma", "neg_scatter", "zero_sigma", "eps_big", "weights", "dims",
                                 "g", "unit", "ndir"])
def test_build_operator_validates(bad):
    _lib()
    prob = problems.make(n=8, ndir=8, eps=0.1)
    if bad == "nan_sigma":
        prob["sigma_t"][3] = np.nan
    elif bad == "neg_scatter":
        prob["sigma_a"][:] = 1e6           # sigma_t/eps - eps*sigma_a < 0
    elif bad == "zero_sigma":
        prob["sigma_t"][0] = 0.0
    elif bad == "eps_big":
        prob["eps"] = 1.5
    elif bad == "weights":
        prob["weights"] = prob["weights"] * 1.01
    elif bad == "dims":
        prob["n"] = (8, 4, 1)
    elif bad == "g":
        prob["g"] = 1.0
    elif bad == "unit":
        prob["dirs"] = prob["dirs"] * 1.1
    elif bad == "ndir":
        prob["dirs"] = np.zeros((0, 3))
        prob["weights"] = np.zeros(0)
    assert _build(prob) == L.RTE_EINVAL


def test_build_operator_rejects_mismatched_model():
    from paper_2604_23265_amd import api
    _lib()
    prob = problems.make(n=8, ndir=8, eps=0.1)
    hdr, t = weights.seeded_weights(2, 16, 16, 2, seed=1)       # 16 directions, not 8
    m = api.Model(weights.pack_mgn1(hdr, t))
    assert _build(prob, m) == L.RTE_EINVAL
    prob2 = problems.make(n=10, ndir=16, eps=0.1)
    hdr, t = weights.seeded_weights(2, 16, 16, 3, seed=1)       # 10 not divisible by 4
    m2 = api.Model(weights.pack_mgn1(hdr, t))
    assert _build(prob2, m2) == L.RTE_EINVAL


def test_null_arguments_are_rejected():
    lib = _lib()
    assert lib.rte_solve(None, None, None, None, 0, None, None, None) == L.RTE_EINVAL
    assert lib.rte_apply(None, None, None, 0, None) == L.RTE_EINVAL
    assert lib.rte_poll(None, 1, None) == L.RTE_EINVAL
    h = C.c_void_p()
    assert lib.rte_server_create(None, 0, 4, C.byref(h)) == L.RTE_EINVAL
    assert lib.rte_prof_enable(99, 1) == L.RTE_EINVAL
    assert lib.rte_build_operator(None, None, None, None, C.byref(h)) == L.RTE_EINVAL
