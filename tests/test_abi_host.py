"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, and its host-only key helpers agree with the oracle's.  No compute
call is made here (there may be no GPU)."""
import ctypes
import itertools

import numpy as np
import pytest

import oracle
import paper_1901_10026_amd as tg


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(tg.library_path())
    names = tg.declared_symbols()
    assert "tg_count" in names and "tg_num_keys" in names
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("L", range(1, 17))
def test_sizes(L):
    assert tg.num_keys(L) == oracle.num_keys(L)
    assert tg.edge_row_width(L) == oracle.row_width(L)


def test_sizes_outside_range_are_zero():
    assert tg.num_keys(0) == 0 and tg.num_keys(17) == 0
    assert tg.edge_row_width(0) == 0


@pytest.mark.parametrize("L", [1, 2, 3, 5, 8, 16])
def test_key_encode_decode_agree_with_oracle(L):
    for shape in range(8):
        k = 3 if shape < 2 else 4
        combos = list(itertools.combinations_with_replacement(range(L), k))
        if len(combos) > 400:
            combos = combos[::len(combos) // 400 + 1] + [combos[-1]]
        for c in combos:
            key = tg.key_encode(L, shape, list(reversed(c)))
            assert key == oracle.key(L, shape, c)
            assert tg.key_decode(L, key) == (shape, tuple(c))


@pytest.mark.parametrize("L", [1, 2, 4, 7])
def test_edge_row_key_agrees_with_oracle(L):
    R = tg.edge_row_width(L)
    for a in range(L):
        for b in range(L):
            for col in range(R):
                assert tg.edge_row_key(L, a, b, col) == oracle.row_key(L, a, b, col)


def test_key_helpers_reject_bad_arguments():
    with pytest.raises(tg.TGError) as e:
        tg.key_encode(3, 0, [0, 1, 3])
    assert e.value.name == "TG_ERR_TYPE_RANGE"
    with pytest.raises(tg.TGError) as e:
        tg.key_decode(3, tg.num_keys(3))
    assert e.value.name == "TG_ERR_INVALID_ARG"
    with pytest.raises(tg.TGError) as e:
        tg.edge_row_key(0, 0, 0, 0)
    assert e.value.name == "TG_ERR_UNSUPPORTED_L"


def test_status_strings():
    lib = tg.lib()
    for code, name in tg.STATUS.items():
        assert lib.tg_status_string(code).decode() == name


def test_count_rejects_arguments_before_touching_the_device():
    lib = tg.lib()
    opt = tg._Options()
    lib.tg_options_default(ctypes.byref(opt))
    dummy = ctypes.c_void_p(8)   # never dereferenced: every call below fails its host checks
    assert lib.tg_count(4, 6, dummy, dummy, dummy, 0, dummy, None, None, ctypes.byref(opt), None) == 4
    assert lib.tg_count(4, 6, dummy, dummy, dummy, 17, dummy, None, None, ctypes.byref(opt), None) == 4
    assert lib.tg_count(4, 6, None, dummy, dummy, 2, dummy, None, None, ctypes.byref(opt), None) == 1
    assert lib.tg_count(4, 6, dummy, dummy, dummy, 2, None, None, None, ctypes.byref(opt), None) == 1
    assert lib.tg_count(4, 5, dummy, dummy, dummy, 2, dummy, None, None, ctypes.byref(opt), None) == 2
    assert lib.tg_count(-1, 6, dummy, dummy, dummy, 2, dummy, None, None, ctypes.byref(opt), None) == 1
    opt.edge_begin, opt.edge_end = 2, 1
    assert lib.tg_count(4, 6, dummy, dummy, dummy, 2, dummy, None, None, ctypes.byref(opt), None) == 1
    opt.edge_begin, opt.edge_end = 0, -1
    opt.schedule = 2   # learned without a model
    assert lib.tg_count(4, 6, dummy, dummy, dummy, 2, dummy, None, None, ctypes.byref(opt), None) == 1
    assert "model" in lib.tg_last_error().decode()


def test_count_global_rejects_arguments_before_touching_the_device():
    lib = tg.lib()
    opt = tg._Options()
    lib.tg_options_default(ctypes.byref(opt))
    dummy = ctypes.c_void_p(8)   # never dereferenced: every call below fails its host checks
    assert lib.tg_count_global(4, 6, dummy, dummy, dummy, 0, dummy, ctypes.byref(opt), None) == 4
    assert lib.tg_count_global(4, 6, dummy, dummy, dummy, 17, dummy, ctypes.byref(opt), None) == 4
    assert lib.tg_count_global(4, 6, dummy, dummy, dummy, 2, None, ctypes.byref(opt), None) == 1
    assert lib.tg_count_global(4, 6, None, dummy, dummy, 2, dummy, ctypes.byref(opt), None) == 1
    assert lib.tg_count_global(4, 5, dummy, dummy, dummy, 2, dummy, ctypes.byref(opt), None) == 2
    assert lib.tg_count_global(-1, 6, dummy, dummy, dummy, 2, dummy, None, None) == 1
    assert lib.tg_count_global_types(4, 6, dummy, dummy, 0, dummy, 2, dummy, None, None, None) == 1
    assert lib.tg_count_global_types(4, 6, dummy, dummy, 2, dummy, 2, None, None, None, None) == 1
    assert lib.tg_count_global_types(4, 6, dummy, dummy, 2, dummy, 0, dummy, None, None, None) == 4


def test_directed_keys_agree_with_the_oracle():
    from oracle import directed as od
    for L in (1, 2, 5, 16):
        assert tg.directed3_num_keys(L) == len(od.keys(L))
    for L in (1, 3):
        ks = od.keys(L)
        for q in range(len(ks)):
            arcs, types = tg.directed3_key_decode(L, q)
            assert arcs | (types[0] << 6) | (types[1] << 10) | (types[2] << 14) == int(ks[q])
            # the key does not depend on the node order
            assert tg.directed3_key_encode(L, arcs, types) == q
    # the 2-path 0 -> 1 -> 2 (types 1, 0, 0) read backwards as 2 -> 1 -> 0
    assert tg.directed3_key_encode(2, 0b010001, [1, 0, 0]) == tg.directed3_key_encode(2, 0b100010, [0, 0, 1])
    with pytest.raises(tg.TGError):
        tg.directed3_key_encode(2, 0b000001, [0, 0, 0])   # one arc: not connected
    lib = tg.lib()
    opt = tg._Options()
    lib.tg_options_default(ctypes.byref(opt))
    dummy = ctypes.c_void_p(8)
    assert lib.tg_count_directed3(4, 6, dummy, dummy, dummy, dummy, 0, dummy, None, None, ctypes.byref(opt), None) == 4
    assert lib.tg_count_directed3(4, 6, dummy, dummy, None, dummy, 2, dummy, None, None, ctypes.byref(opt), None) == 1
    assert lib.tg_count_directed3(4, 6, dummy, dummy, dummy, dummy, 2, None, None, None, ctypes.byref(opt), None) == 1
    assert lib.tg_count_directed3(4, 5, dummy, dummy, dummy, dummy, 2, dummy, None, None, ctypes.byref(opt), None) == 2


def test_type_permutations_keep_type_frequencies():
    types = np.array([0, 1, 1, 2, 2, 2, 3], np.uint8)
    perms = tg.type_permutations(types, 5, seed=9)
    assert perms.shape == (5, 7)
    for p in perms:
        assert np.array_equal(np.sort(p), types)
    assert np.array_equal(perms, tg.type_permutations(types, 5, seed=9))
    assert not np.array_equal(perms, tg.type_permutations(types, 5, seed=10))


def test_tuning_defaults_and_round_trip():
    t = tg.Tuning.default()
    assert t.tlist_budget_mib == 16384 and t.clique_lds_ids == 4096
    # the last fields land where the library writes them (same layout)
    assert t.c4_parts == 1 and t.tau_hub_min_degree == 4096 and t.c4_split_log2 == 32
    d = t.as_dict()
    d["tlist_budget_mib"] = 0
    assert tg.Tuning.from_dict(d).as_dict() == d


def test_directed4_keys_match_the_oracle():
    """The library's directed 4-node key list (host tables, no device work)
    equals the oracle's: same count and the same canonical digraph per key."""
    import paper_1901_10026_amd as tg
    from oracle import directed4 as d4
    assert tg.directed4_num_keys(0) == 0 and tg.directed4_num_keys(5) == 0
    for L in (1, 2, 3):
        ks = d4.keys(L)
        assert tg.directed4_num_keys(L) == len(ks)
        for q in list(range(0, len(ks), max(1, len(ks) // 300))) + [len(ks) - 1]:
            arcs, ty = tg.directed4_key_decode(L, q)
            assert arcs | sum(t << (12 + 4 * p) for p, t in enumerate(ty)) == int(ks[q])
