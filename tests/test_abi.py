"""Host-side checks of the C ABI: the library loads, exports every declared call,
validates arguments before touching a device, and generates per-robot code. No GPU."""
import os
import re

import numpy as np
import pytest

from paper_2109_06976_amd import grid, synth

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "grid.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(grid_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = grid.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(grid.EXPORTED)


def test_status_strings():
    assert grid.status_string(0) == "GRID_OK"
    assert grid.status_string(-1) == "GRID_EINVAL"
    assert grid.status_string(-5) == "GRID_ECOMPILE"
    assert grid.status_string(17) == "GRID_UNKNOWN"


def _bad(robot, **changes):
    r = robot.copy()
    for k, v in changes.items():
        setattr(r, k, v)
    return r


@pytest.mark.parametrize("mutate,status", [
    (lambda r: _bad(r, parent=np.array([-1, 0, 2, 2, 3, 4, 5], np.int32)), grid.GRID_EINVAL),
    (lambda r: _bad(r, mass=np.where(np.arange(7) == 3, -1.0, r.mass)), grid.GRID_EINVAL),
    (lambda r: _bad(r, E_T=r.E_T * 2.0), grid.GRID_EINVAL),
    (lambda r: _bad(r, Ic=np.tile([0.1, 0.1, 0.1, 0.5, 0, 0], (7, 1))), grid.GRID_EINVAL),
    (lambda r: _bad(r, r=np.where(np.arange(21).reshape(7, 3) == 4, np.nan, r.r)),
     grid.GRID_EINVAL),
])
def test_model_create_rejects_bad_descriptions_before_device_work(mutate, status):
    with pytest.raises(grid.GridError) as e:
        grid.Model(mutate(synth.chain7()))
    assert e.value.status == status


def test_model_create_rejects_too_many_bodies():
    robot = synth.random_model(synth.chain_parent(33), 0)
    with pytest.raises(grid.GridError) as e:
        grid.Model(robot)
    assert e.value.status == grid.GRID_EUNSUPPORTED


def test_unknown_flags_rejected():
    with pytest.raises(grid.GridError) as e:
        grid.Model(synth.chain7(), flags=8)
    assert e.value.status == grid.GRID_EINVAL


def _table(src, name):
    m = re.search(name + r"\[\d+\] = \{([^}]*)\}", src)
    return [int(x.replace("ull", ""), 0) for x in m.group(1).split(",")]


def test_codegen_tables_quadruped():
    src = grid.codegen_source(synth.quadruped_parent())
    assert "#define GRID_N 12" in src and "#define GRID_NLEV 3" in src
    assert "#define GRID_L 32" in src
    levels = _table(src, "kLevelMask")
    assert levels == [0b001001001001, 0b010010010010, 0b100100100100]
    # two inward rounds (level 2 -> 1, level 1 -> 0); each leg has one child per level
    assert _table(src, "kRoundMask") == [0b100100100100, 0b010010010010]
    assert _table(src, "kBranch") == [0, 0, 0, 3, 3, 3, 6, 6, 6, 9, 9, 9]


def test_codegen_rounds_have_distinct_parents():
    parent = synth.humanoid_parent("anatomical")
    src = grid.codegen_source(parent)
    rounds = _table(src, "kRoundMask")
    seen = 0
    for mask in rounds:
        bodies = [i for i in range(30) if mask >> i & 1]
        parents = [parent[i] for i in bodies]
        assert len(set(parents)) == len(parents)
        assert all(p >= 0 for p in parents)
        assert seen & mask == 0
        seen |= mask
    # every non-root body adds into its parent exactly once
    assert seen == sum(1 << i for i in range(30) if parent[i] >= 0)
    # body 1 (second torso link) has three children at the same level: three rounds there
    assert "#define GRID_NLEV 9" in src


def test_codegen_related_masks():
    parent = synth.humanoid_parent("anatomical")
    rel = _table(grid.codegen_source(parent), "kRelated")
    anc = [set() for _ in range(30)]
    for i in range(30):
        a = parent[i]
        while a >= 0:
            anc[i].add(a)
            a = parent[a]
    for i in range(30):
        for k in range(30):
            expect = i == k or k in anc[i] or i in anc[k]
            assert bool(rel[i] >> k & 1) == expect


def test_codegen_rejects_bad_topology():
    with pytest.raises(grid.GridError) as e:
        grid.codegen_source(np.array([-1, 1], np.int32))
    assert e.value.status == grid.GRID_EINVAL
