"""The C-ABI library loads, exports every declared symbol, and its host-only planner
matches the reference split.  No device calls."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from oracle import plan
from paper_2009_04755_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2009_04755_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    header = open(os.path.join(ROOT, "include", "rocket.h")).read()
    declared = set(re.findall(r"\b(rocket_[a-z_]+)\s*\(", header))
    assert declared == set(_lib.SYMBOLS)
    for name in declared:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code, name in [(0, "ROCKET_OK"), (-1, "ROCKET_E_INVALID"), (-5, "ROCKET_E_KEYRANGE"), (-6, "ROCKET_E_UNSORTED")]:
        assert lib.rocket_status_str(code).decode() == name


@pytest.mark.parametrize("n,T", [(0, 4), (1, 4), (2, 1), (8, 1), (17, 4), (257, 64), (300, 7), (4096, 256)])
def test_native_planner_matches_reference(lib, n, T):
    from paper_2009_04755_amd import api
    assert api.plan_tiles(n, T) == plan.quadtree_leaves(n, T)


def test_native_pair_index(lib):
    n = 37
    pi, pj = oracle.all_pairs(n)
    got = [lib.rocket_pair_index(int(i), int(j), n) for i, j in zip(pi, pj)]
    assert got == list(range(pi.size))
    assert lib.rocket_pair_index(4978, 4979, 4980) == 12397710 - 1


def test_bad_arguments_rejected_without_device(lib):
    assert lib.rocket_plan_tiles(-1, 4, None, None, 0) < 0
    assert lib.rocket_plan_tiles(5, 0, None, None, 0) < 0
    st = lib.rocket_prepare(None, None, 4, 3, None)
    assert st == _lib.E_INVALID


def test_binding_matches_header_enums_and_items():
    header = open(os.path.join(ROOT, "include", "rocket.h")).read()
    end = header.index("} rocket_pair_fn;")
    enum = header[header.rindex("typedef enum {", 0, end):end]
    enum = re.sub(r"/\*.*?\*/", "", enum, flags=re.S)
    fns = dict((k, int(v)) for k, v in re.findall(r"ROCKET_(\w+) = (\d+)", enum))
    assert {k.lower(): v for k, v in fns.items()} == _lib.FN_BY_NAME
    opts = dict((k.lower(), int(v)) for k, v in re.findall(r"ROCKET_OPT_(\w+) = (\d+)", header))
    assert opts == _lib.OPT
    body = re.search(r"typedef struct \{(.*?)\} rocket_items;", header, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"(\w+);", body)
    assert fields == [f for f, _ in _lib.Items._fields_]
