"""The C ABI without a GPU: the library loads, exports every symbol that
include/sg.h declares, rejects bad arguments synchronously (before any HIP
call), and its chunk plan tiles the requested mask range."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sg.h")


@pytest.fixture(scope="module")
def L():
    from paper_1904_03621_amd import _lib
    return _lib


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(sg_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_binding_exports(L):
    assert _declared_functions() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    lib = L.lib()
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match(L):
    import paper_1904_03621_amd as pkg
    for name in _declared_functions():
        if name in ("sg_last_error",):
            continue
        assert hasattr(pkg, name) or hasattr(L, name), name


@pytest.mark.parametrize("case", [
    dict(N=0), dict(N=64), dict(S=0), dict(S=(1 << 20) + 1), dict(N=4, S=17),
    dict(lo=10), dict(lo=64, hi=64), dict(hi=(1 << 20) + 64, N=20), dict(lo=0, hi=100, N=20),
    dict(lo=128, hi=192, S=65, N=20), dict(null=True),
])
def test_validation_is_synchronous(L, case):
    lib = L.lib()
    N = case.get("N", 20)
    S = case.get("S", 10)
    lo = case.get("lo", 0)
    hi = case.get("hi", 1 << N if 0 < N <= 63 else 64)
    p = 0 if case.get("null") else 4096  # never dereferenced: validation fails first
    if "lo" in case or "hi" in case:
        st = lib.sg_low_spectrum_range_f32(N, p, p, S, lo, hi, p, p, 0)
        st2 = lib.sg_low_spectrum_range_i32(N, p, p, S, lo, hi, p, p, 0)
    else:
        st = lib.sg_low_spectrum_f32(N, p, p, S, p, p, 0)
        st2 = lib.sg_low_spectrum_i32(N, p, p, S, p, p, 0)
    assert st == L.SG_EINVAL and st2 == L.SG_EINVAL
    assert L.last_error() != ""


@pytest.mark.parametrize("case", [
    dict(B=0), dict(N=6), dict(N=41), dict(nb=0), dict(nb=5), dict(S=0), dict(S=4097),
    dict(S=129, N=7), dict(null=True),
])
def test_batched_and_logz_validation_is_synchronous(L, case):
    lib = L.lib()
    B, N, S, nb = case.get("B", 4), case.get("N", 20), case.get("S", 8), case.get("nb", 3)
    p = 0 if case.get("null") else 4096  # never dereferenced: validation fails first
    st = lib.sg_logz_forward_f32(B, N, p, p, nb, p, S, p, p, p, p, 0)
    assert st == L.SG_EINVAL and L.last_error() != ""
    if "S" not in case:
        st = lib.sg_logz_backward_f32(B, N, p, p, nb, p, p, p, p, p, p, 0)
        assert st == L.SG_EINVAL and L.last_error() != ""
        st = lib.sg_logz_backward_noalloc_f32(B, N, p, p, nb, p, p, p, p, p, p, 0)
        assert st == L.SG_EINVAL and L.last_error() != ""
    if "nb" not in case and not (N == 7 and S == 129):
        st = lib.sg_low_spectrum_batched_f32(B, p, N, p, p, S, p, p, 0)
        assert st == L.SG_EINVAL and L.last_error() != ""


@pytest.mark.parametrize("case", [dict(N=0), dict(N=64), dict(n_bins=0), dict(n_bins=8193),
                                  dict(null=True)])
def test_dos_validation_is_synchronous(L, case):
    lib = L.lib()
    N, n_bins = case.get("N", 12), case.get("n_bins", 100)
    p = 0 if case.get("null") else 4096  # never dereferenced: validation fails first
    assert lib.sg_density_of_states_i32(N, p, p, -50, n_bins, p, 0) == L.SG_EINVAL
    assert L.last_error() != ""
    if "n_bins" not in case:
        assert lib.sg_energy_bound_i32(N, p, p, p, 0) == L.SG_EINVAL


@pytest.mark.parametrize("args", [(0, 20, 8), (4, 0, 8), (4, 64, 8), (4, 20, 0),
                                  (4, 20, (1 << 20) + 1)])
def test_reserve_validation(L, args):
    assert L.lib().sg_reserve(*args, 0) == L.SG_EINVAL


def _check_plan(L, N, S, lo, hi, fill):
    plan = L.sg_debug_plan(N, S, lo, hi, fill)
    assert plan, "empty plan"
    cur = lo
    nmax = min(22, N)
    first_states = None
    for (first, n, lanes) in plan:
        assert first == cur, "chunks must tile the range in ascending order"
        # n = 0: a range end shorter than a 128-state block, one thread per state
        assert n == 0 or 7 <= n <= nmax
        assert n > 0 or lanes < 256
        assert first % (1 << n) == 0, "prefix base must be whole"
        assert lanes >= 1
        size = lanes << n
        if first_states is None:
            first_states = size
        cur += size
    assert cur == hi
    return plan, first_states


@pytest.mark.parametrize("N,S,lo,hi,fill", [
    (24, 100, 0, 1 << 24, 1 << 19),
    (48, 1000, 0, 1 << 48, 1 << 19),
    (48, 10000, 0, 1 << 48, 1 << 19),
    (48, 1000, 0, 1 << 48, 5 * 256 * 256),   # occupancy 5 -> non power of two fill
    (30, 64, 64 * 12345, 64 * 9999999, 1 << 19),
    (32, 7, (1 << 31), (1 << 31) + (1 << 25), 1 << 19),
    (6, 1, 0, 64, 1 << 19),
    (10, 1024, 0, 1024, 64),
    (40, 1 << 20, 0, 1 << 40, 1 << 19),
    (63, 100, (1 << 63) - (1 << 44), 1 << 63, 1 << 19),   # the largest N, top of the space
    (63, 64, (1 << 62) + 64 * 777, (1 << 62) + (1 << 33), 1 << 19),
])
def test_plan_tiles_range(L, N, S, lo, hi, fill):
    plan, first = _check_plan(L, N, S, lo, hi, fill)
    # the first chunk runs without a threshold: it holds at least S states
    # (and every later chunk at most as many states as all earlier ones
    # together, except the fixed-size tail)
    assert first >= min(S, hi - lo)
    done = 0
    big = fill << min(22, N)
    for (first_m, n, lanes) in plan[1:]:
        done = first_m - lo
        size = lanes << n
        assert size <= max(done, big)


def test_plan_uses_full_fill_at_scale(L):
    fill = 1 << 19
    plan = L.sg_debug_plan(48, 1000, 0, 1 << 48, fill)
    big = [c for c in plan if c[1] == 22]
    assert len(big) >= 100
    # every chunk of the second half of the space runs a full device
    assert all(l == fill for (m, _, l) in plan if m >= (1 << 47))
    assert len(plan) < 200


def test_run_info_struct_matches_header(L):
    """The ctypes mirror of sg_run_info lists the header's fields in order."""
    import re
    text = open(os.path.join(ROOT, "include", "sg.h")).read()
    body = text[text.index("typedef struct"):text.index("} sg_run_info;")]
    names = re.findall(r"^\s*(?:int64_t|int32_t|double|float)\s+(\w+);", body, re.M)
    assert names == [n for n, _ in L.RunInfo._fields_]
