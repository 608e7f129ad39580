"""Host-side tests of the C ABI (no GPU): exported symbols, the einsum parser,
and argument validation that must fail before anything is enqueued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dn():
    import paper_2206_08301_amd as m
    m._lib.load()
    return m


def test_library_exports_every_declared_symbol(dn):
    header = open(os.path.join(ROOT, "include", "deinsum.h")).read()
    declared = set(re.findall(r"^(?:deinsum_status|void|const char\s*\*)\s*(deinsum_\w+)\s*\(", header, re.M))
    assert declared == set(dn._lib.EXPORTS)
    lib = dn._lib.load()
    for name in declared:
        assert hasattr(lib, name), name


def test_version(dn):
    assert "gfx950" in dn.version()


TAB4 = {
    "ijk,ja,ka->ia": (1, 3, 0, [1, 2]),
    "ijk,ia,ka->ja": (1, 3, 1, [0, 2]),
    "ijk,ia,ja->ka": (1, 3, 2, [0, 1]),
    "ijklm,ja,ka,la,ma->ia": (1, 5, 0, [1, 2, 3, 4]),
    "ijklm,ia,ja,la,ma->ka": (1, 5, 2, [0, 1, 3, 4]),
    "ijklm,ia,ja,ka,la->ma": (1, 5, 4, [0, 1, 2, 3]),
    "ijklm,jb,kc,ld,me->ibcde": (2, 5, 0, [1, 2, 3, 4]),
}


@pytest.mark.parametrize("spec", sorted(TAB4))
def test_parse_tab4_strings(dn, spec):
    s = dn.parse(spec)
    kind, order, free, fm = TAB4[spec]
    assert (s.kind, s.order, s.free_mode) == (kind, order, free)
    assert list(s.factor_mode)[: order - 1] == fm
    assert s.out_idx.decode() == spec.split("->")[1]


def test_parse_operand_order_and_whitespace(dn):
    s = dn.parse(" ijk , ka , ja -> ia ")
    assert s.kind == 1 and s.free_mode == 0
    assert list(s.factor_mode)[:2] == [2, 1]
    assert list(s.operand_of_mode)[:3] == [-1, 1, 0]


def test_parse_ttmc_other_modes(dn):
    s = dn.parse("ijk,ib,kc->bjc")
    assert s.kind == 2 and s.free_mode == 1
    s = dn.parse("ij,ia->aj")
    assert s.kind == 2 and s.free_mode == 1
    s = dn.parse("ij,ja->ia")
    assert s.kind == 1  # order 2: the MTTKRP and TTMc outputs coincide


def test_parse_mttkrp_gemm_chain(dn):
    """The MTTKRP followed by a matrix product (the paper's running example)."""
    s = dn.parse("ijk,ja,ka,al->il")
    assert s.kind == 3 and s.order == 3 and s.free_mode == 0 and s.n_factors == 2
    s = dn.parse(" ijkl , ia , ka , la , ab -> jb ")
    assert s.kind == 3 and s.free_mode == 1 and list(s.factor_mode[:3]) == [0, 2, 3]


@pytest.mark.parametrize("bad,status", [
    ("ijk,ja,ka", -2),            # implicit output
    ("...k,ka->...a", -2),        # ellipsis
    ("iik,ia,ka->ia", -2),        # repeated letter (diagonal)
    ("ijk,j1,ka->ia", -2),        # non-letter
    ("ijk,,ka->ia", -2),          # empty operand
    ("ijk,aj,ka->ia", -3),        # transposed factor
    ("ijk,ja,ka->ai", -3),        # output permuted
    ("ijk,ia,ja,ka->ia", -3),     # factor on the free mode / too many factors
    ("ijk,ja,ja->ia", -3),        # mode contracted twice
    ("ijk,ja->ia", -3),           # a mode neither free nor contracted
    ("ijk,ja,kb->ia", -3),        # mixed rank letters, MTTKRP output
    ("ijk,jb,kc->icb", -3),       # TTMc output not in place
    ("i,ia->a", -3),              # order 1
    ("abcdefghi,ba,cz,dz,ez,fz,gz,hz,iz->az", -3),  # order 9
    ("ijk,jaa,ka->ia", -2),
    ("ijk,ja,ka,bl->il", -3),     # chain matrix not indexed by the rank letter
    ("ijk,ja,ka,aj->ij", -3),     # chain letter taken from X
    ("ijk,ja,ka,al->li", -3),     # chain output permuted
    ("ijk,jb,kc,bl->il", -3),     # chain after TTMc-style factors
    ("ijk,ja,ka,aa->ia", -2),     # repeated letter in the chain matrix
])
def test_parse_rejects(dn, bad, status):
    with pytest.raises(dn.DeinsumError) as e:
        dn.parse(bad)
    assert e.value.status == status
    assert dn.last_error()


def test_workspace_size_host_only(dn):
    n = dn.workspace_size("ijk,ja,ka->ia", [1024, 1024, 1024], [24])
    assert 0 < n < 0.02 * 8 * 1024 ** 3
    n2 = dn.workspace_size("ijk,ia,ja->ka", [1024, 1024, 1024], [24])
    assert 0 < n2 < 0.02 * 8 * 1024 ** 3
    n3 = dn.workspace_size("ijk,jb,kc->ibc", [1024, 1024, 1024], [32, 32])
    assert 0 < n3 < 0.02 * 8 * 1024 ** 3


def _call_mttkrp(dn, spec, dims, R, X, U, M, opts=None):
    lib = dn._lib.load()
    s = dn.parse(spec)
    d = (ctypes.c_int64 * len(dims))(*dims)
    ptrs = (ctypes.c_void_p * len(U))(*U)
    return lib.deinsum_mttkrp(ctypes.byref(s), d, R, X, ptrs, M,
                              ctypes.byref(opts) if opts is not None else None, None)


def test_mttkrp_argument_errors_before_enqueue(dn):
    # Fake (never dereferenced) addresses: validation must reject before any launch.
    X, B, C, M = 0x10000000, 0x20000000, 0x30000000, 0x40000000
    assert _call_mttkrp(dn, "ijk,ja,ka->ia", [4, 4, 4], 0, X, [B, C], M) == -4       # R < 1
    assert _call_mttkrp(dn, "ijk,ja,ka->ia", [4, 4, 4], 300, X, [B, C], M) == -4     # R > 256
    assert _call_mttkrp(dn, "ijk,ja,ka->ia", [4, -1, 4], 2, X, [B, C], M) == -4      # negative dim
    assert _call_mttkrp(dn, "ijk,ja,ka->ia", [4, 4, 4], 2, X, [B, None], M) == -1    # null factor
    assert _call_mttkrp(dn, "ijk,ja,ka->ia", [4, 4, 4], 2, X, [B, C], X + 8) == -1   # M overlaps X
    assert _call_mttkrp(dn, "ijk,ja,ka->ia", [4, 4, 4], 2, X, [B, C], B) == -1       # M overlaps a factor
    o = dn._lib.Opts()
    dn._lib.load().deinsum_opts_init(ctypes.byref(o))
    o.precision = 9
    assert _call_mttkrp(dn, "ijk,ja,ka->ia", [4, 4, 4], 2, X, [B, C], M, o) == -1    # bad precision
    o.precision = 0
    o.out_dtype = 1
    assert _call_mttkrp(dn, "ijk,ja,ka->ia", [4, 4, 4], 2, X, [B, C], M, o) == -1    # FP64 form, F32 out
    lib = dn._lib.load()
    s = dn.parse("ijk,jb,kc->ibc")
    d = (ctypes.c_int64 * 3)(4, 4, 4)
    assert lib.deinsum_mttkrp(ctypes.byref(s), d, 2, X, (ctypes.c_void_p * 2)(B, C), M, None, None) == -1  # TTMc spec


def test_mttkrp_gemm_chain_argument_errors_before_enqueue(dn):
    # Fake (never dereferenced) addresses: validation must reject before any launch.
    X, B, C, D, Y = 0x10000000, 0x20000000, 0x30000000, 0x50000000, 0x60000000
    lib = dn._lib.load()
    s = dn.parse("ijk,ja,ka,al->il")
    d = (ctypes.c_int64 * 3)(4, 4, 4)
    U = (ctypes.c_void_p * 2)(B, C)
    call = lambda R, L, Dp, Yp, spec=s: lib.deinsum_mttkrp_mm(ctypes.byref(spec), d, R, L, X, U, Dp, Yp, None, None)
    assert call(0, 3, D, Y) == -4            # R < 1
    assert call(2, 0, D, Y) == -4            # L < 1
    assert call(2, 5000, D, Y) == -4         # L too large
    assert call(2, 3, None, Y) == -1         # null C
    assert call(2, 3, D, D + 8) == -1        # Y overlaps C
    assert call(2, 3, D, X + 8) == -1        # Y overlaps X
    assert call(2, 3, D, B) == -1            # Y overlaps a factor
    assert call(2, 3, D, Y, dn.parse("ijk,ja,ka->ia")) == -1  # not a chain spec
    assert dn.last_error()


def test_ttmc_rank_limit(dn):
    with pytest.raises(dn.DeinsumError):
        dn.workspace_size("ijk,jb,kc->ibc", [8, 8, 8], [65, 4])


def test_synth_and_convert_argument_errors(dn):
    lib = dn._lib.load()
    assert lib.deinsum_synth_fill(None, 0, 10, 1, 0, 0, None) == -1
    assert lib.deinsum_synth_fill(ctypes.c_void_p(0x1000), 0, 10, 1, 0, 7, None) == -1
    assert lib.deinsum_synth_fill(None, 0, 0, 1, 0, 0, None) == 0  # nothing to do
    assert lib.deinsum_convert(ctypes.c_void_p(0x1000), 0, ctypes.c_void_p(0x1008), 1, 10, None) == -1


# ---------------------------------------------------------------- autotuner plan cache (host side)
KEY_1024_M0 = "s:N3:n0:p0:R24:1024x1024x1024"


def test_tune_cache_drives_the_planner(dn, tmp_path):
    spec, dims = "ijk,ja,ka->ia", [1024, 1024, 1024]
    dn.tune_clear()
    heuristic = dn.workspace_size(spec, dims, [24])
    forced = dn.workspace_size(spec, dims, [24], split_hint=1)  # hints bypass the cache
    assert forced < heuristic
    f = tmp_path / "cache.txt"
    f.write_text(f"# comment\n{KEY_1024_M0} 2 16 1 0 1 0 0 123.5\n")
    dn.tune_load(f)
    assert dn.tune_entries() == 1
    assert dn.workspace_size(spec, dims, [24]) == forced
    assert dn.workspace_size(spec, dims, [24], split_hint=4) != forced
    out = tmp_path / "saved.txt"
    dn.tune_save(out)
    assert f"{KEY_1024_M0} 2 16 1 0 1 0 0 123.5" in out.read_text()
    dn.tune_clear()
    assert dn.tune_entries() == 0
    assert dn.workspace_size(spec, dims, [24]) == heuristic


def test_tune_cache_stale_variant_falls_back(dn, tmp_path):
    spec, dims = "ijk,ja,ka->ia", [1024, 1024, 1024]
    dn.tune_clear()
    heuristic = dn.workspace_size(spec, dims, [24])
    f = tmp_path / "stale.txt"
    f.write_text(f"{KEY_1024_M0} 2 99 1 0 1 0 0 1.0\n")
    dn.tune_load(f)
    assert dn.workspace_size(spec, dims, [24]) == heuristic
    dn.tune_clear()


def test_tune_cache_mode0_through_ttmc(dn, tmp_path):
    """Order-3 mode 0 (FP64, large): by default through the fused TTMc pass; a cache entry
    with order 2 names its variant (a variant no longer compiled falls back to the default
    one); an entry for a stream kernel selects that kernel's smaller workspace."""
    spec, dims = "ijk,ja,ka->ia", [1024, 1024, 1024]
    dn.tune_clear()
    default = dn.workspace_size(spec, dims, [24])
    stream = dn.workspace_size(spec, dims, [24], split_hint=1)  # a hint keeps the stream kernel
    assert default > stream  # the TTMc pass holds R x R tiles and a padded factor copy
    f = tmp_path / "ttmc.txt"
    for line, want in ((f"{KEY_1024_M0} 1 1 1 0 2 2 0 1.0\n", default), (f"{KEY_1024_M0} 1 1 1 0 99 2 0 1.0\n", default),
                       (f"{KEY_1024_M0} 2 16 1 0 1 0 0 1.0\n", stream)):
        f.write_text(line)
        dn.tune_clear()
        dn.tune_load(f)
        assert dn.workspace_size(spec, dims, [24]) == want, line
    dn.tune_clear()


def test_tune_rejects_bad_input(dn, tmp_path):
    f = tmp_path / "bad.txt"
    f.write_text("s:N3:n0:p0:R24:8x8x8 two 16 1 0 1 0 0 1.0\n")
    with pytest.raises(dn.DeinsumError) as e:
        dn.tune_load(f)
    assert e.value.status == -2
    with pytest.raises(dn.DeinsumError):
        dn.tune_load(tmp_path / "missing.txt")
    lib = dn._lib.load()
    s = dn.parse("ijk,ja,ka->ia")
    d = (ctypes.c_int64 * 3)(8, 8, 8)
    ptrs = (ctypes.c_void_p * 2)(None, None)
    for fn in (lib.deinsum_tune_mttkrp, lib.deinsum_tune_batch_mttkrp):
        assert fn(ctypes.byref(s), d, 4, None, ptrs, None, None, 0, None, None) == -1  # reps = 0
    dn.tune_clear()


def test_row_walk_plan_hint_host(dn):
    """plan_hint 3 (order-3 mode 0, reduced forms) plans without a GPU; other modes, other
    orders and the FP64 form reject it."""
    ws = dn.workspace_size("ijk,ja,ka->ia", (40, 70, 200), [24], "fp32", plan_hint=3)
    # FP32 slices of 128 along mode 2: 2 FP64 partials of 40 rows x 32 columns, then U^1 in FP32
    # packed per 16-row tile (5 tiles) and lane: 5 x 64 lanes x 4 rows x 2 column tiles
    assert ws == 2 * 40 * 32 * 8 + 5 * 64 * 4 * 2 * 4
    for spec, dims, prec in (("ijk,ia,ka->ja", (40, 70, 200), "fp32"), ("ijk,ja,ka->ia", (40, 70, 200), "fp64"),
                             ("ijkl,ja,ka,la->ia", (8, 9, 10, 11), "fp32")):
        with pytest.raises(dn.DeinsumError) as e:
            dn.workspace_size(spec, dims, [24], prec, plan_hint=3)
        assert e.value.status == -3


def test_tune_cache_row_walk_entry(dn, tmp_path):
    """Order-3 mode 0 in a reduced form: the default for far-apart rows is the row walk;
    a cache entry with order 3 names a row-walk kernel and its chunk count, one with a
    stream-kernel order keeps the K-contiguous kernel, and an entry for a row-walk
    variant that is not compiled falls back to the heuristic."""
    spec, dims = "ijk,ja,ka->ia", [1024, 1024, 1024]
    key = "s:N3:n0:p1:R24:1024x1024x1024"  # FP32
    dn.tune_clear()
    default = dn.workspace_size(spec, dims, [24], "fp32")
    walk = dn.workspace_size(spec, dims, [24], "fp32", plan_hint=3)
    assert default == walk  # 1024^3 FP32: rows 4 MiB apart, the walk by default
    # row walk with 8 chunks: FP32 slices of 128 -> 8 slices of 1024 rows x 32 columns
    # in FP64, then U^1 packed in FP32 (64 tiles x 64 lanes x 4 rows x 2 column tiles)
    f = tmp_path / "walk.txt"
    f.write_text(f"{key} 2 32 1 0 8 3 0 1.0\n")
    dn.tune_load(f)
    assert dn.workspace_size(spec, dims, [24], "fp32") == 8 * 1024 * 32 * 8 + 64 * 64 * 4 * 2 * 4
    f.write_text(f"{key} 2 32 1 0 4 0 0 1.0\n")  # the K-contiguous kernel, 4 chunks
    dn.tune_clear()
    dn.tune_load(f)
    kc = dn.workspace_size(spec, dims, [24], "fp32")
    assert kc == dn.workspace_size(spec, dims, [24], "fp32", plan_hint=1, split_hint=4)
    f.write_text(f"{key} 2 99 1 0 8 3 0 1.0\n")  # no such row-walk variant
    dn.tune_clear()
    dn.tune_load(f)
    assert dn.workspace_size(spec, dims, [24], "fp32") == default
    dn.tune_clear()
