"""The C-ABI library loads on a machine without a GPU and exports every
symbol include/aop.h declares; host-side validation and workspace sizing
(no device calls) behave as documented."""
import ctypes
import os
import re

import pytest

from paper_2303_02317_amd import binding, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "aop.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(aop_[a-z_]+)\s*\(", src)))


def test_header_lists_match_binding():
    assert declared_functions() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.aop_version()


def test_status_strings():
    lib = binding.load()
    for code in range(8):
        assert lib.aop_status_str(code)


@pytest.mark.parametrize("bad,code", [
    (dict(S0=-1.0), 1), (dict(K=0.0), 1), (dict(sigma=0.0), 1), (dict(expiry=float("nan")), 1),
    (dict(T=0), 1), (dict(T=(1 << 21) + 1), 5), (dict(model=7), 1), (dict(q=-0.01), 1),
])
def test_validation(bad, code):
    o = dict(inputs.CONFIG1)
    o.update(bad)
    assert binding.validate(o) == code


def test_validation_model_specific():
    o = dict(inputs.CONFIG1, model=2)  # BSM put needs q = 0
    assert binding.validate(o) == 1
    o["q"] = 0.0
    assert binding.validate(o) == 0
    # p > 1: the up move cannot cover the growth at T = 1
    assert binding.validate(dict(inputs.CONFIG1, r=0.9, q=0.0, sigma=0.01, T=1)) == 2
    # a trinomial call with R < 0 is outside the hypotheses of the Sec. 3 lemmas;
    # the binomial call and the BSM put accept it
    assert binding.validate(dict(inputs.CONFIG1, model=1, r=-0.01, q=0.0)) == 2
    assert binding.validate(dict(inputs.CONFIG1, model=0, r=-0.01, q=0.0)) == 0
    assert binding.validate(dict(inputs.CONFIG1, model=2, r=-0.01, q=0.0)) == 0


def test_workspace_bytes_grow_with_T():
    a = binding.workspace_bytes(inputs.batch(2, 10, 4, 0))
    b = binding.workspace_bytes(inputs.batch(2, 14, 4, 0))
    assert 0 < a < b
    # invalid options take no workspace
    bad = [dict(inputs.CONFIG1, S0=-1.0)]
    # descriptor, counters and the work pool of the persistent kernel only
    assert binding.workspace_bytes(bad) == binding.workspace_bytes([])
    assert binding.workspace_bytes([]) <= 9 * 2**20
