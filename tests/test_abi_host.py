"""C ABI on a machine without a GPU: the library loads, exports every
declared entry point, validates its inputs, and its host-side setup (block
split, S~ of eq. (7), SA-AMG of Section 3.3) reproduces the oracle's
hierarchy level by level (handles built with MDP_HOST_ONLY, no device)."""

import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from hierfile_util import to_version_1
from oracle import amg, blocks as ob
from oracle import assembly as oa
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mdp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mdp_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 18
    for name in names:
        assert hasattr(L.lib, name), name
    assert set(names) == set(L.EXPORTED)


def test_options_default_values():
    o = L.mdp_options_default()
    assert (o.precision, o.vcycles, o.pre_sweeps, o.post_sweeps) == (L.MDP_FP64, 1, 1, 1)
    assert (o.strength_theta, o.max_coarse, o.max_dense, o.max_levels) == (0.02, 400, 2000, 10)
    assert (o.restart, o.max_iter, o.rtol, o.flags) == (64, 1000, 1e-8, 0)
    assert o.block_form == L.MDP_BLOCK_LOWER
    assert L.mdp_version().startswith("mdp")


def _host_handle(A, part, **kw):
    o = L.mdp_options_default(flags=L.MDP_HOST_ONLY, **kw)
    return L.mdp_setup(A, part, o)


def _csr(h, block, level, mat):
    ptr, col, val, shape = L.mdp_level_export(h, block, level, mat)
    return sp.csr_matrix((val, col, ptr), shape=shape)


SCEN = [
    lambda: synth.grid_2d_four_lines(32),
    lambda: synth.regular_3d(n=12, seed=3),
    lambda: synth.regular_3d(n=10, k_par=1e-4, kappa=1e4, seed=5),
    lambda: synth.random_2d(4, n_range=(40, 60)),
    lambda: synth.tiny_3d(9, seed=2),
]


def _flux(assemble):
    def f(sc):
        out = assemble(sc)
        return out[0], out[1], out[2]
    return f


@pytest.mark.parametrize("form", ["pressure", "flux", "flux-labeled"])
@pytest.mark.parametrize("make", SCEN)
def test_host_hierarchy_matches_oracle(make, form):
    """Both block readings: the primal pressure system, and the paper's
    own with interface fluxes as Gamma (oracle/mixed_dim.py), the latter also
    with dimension-aware aggregation (mdp_setup_labeled)."""
    from oracle import mixed_dim as md
    from paper_2206_03203_amd import tpfa_flux
    sc = make()
    labels = None
    if form == "pressure":
        A, b, part = tpfa.assemble(sc)
    else:
        A, b, part, finfo = tpfa_flux.assemble_flux(sc)
        if form == "flux-labeled":
            labels = finfo["labels"]
    opts = amg.AMGOptions(max_coarse=40)
    h = L.mdp_setup(A, part, L.mdp_options_default(flags=L.MDP_HOST_ONLY, max_coarse=40), labels=labels)
    try:
        if form == "pressure":
            Ao, bo, po = oa.assemble(sc)
        else:
            Ao, bo, po, oinfo = md.assemble_flux(sc)
            assert labels is None or np.array_equal(labels, oinfo["labels"])
        omega, gamma, Aoo, Aog, Ago, Agg = ob.split(Ao, po)
        S = ob.approx_schur(Aoo, Aog, Ago, Agg)
        info = L.mdp_info(h)
        assert info["n_omega"] == Aoo.shape[0] and info["n_gamma"] == Agg.shape[0]
        for block, M, idx in ((L.MDP_BLOCK_OMEGA, S, omega), (L.MDP_BLOCK_GAMMA, Agg, gamma)):
            H = amg.setup(M, opts, None if labels is None else labels[idx])
            nl = info["levels_omega" if block == L.MDP_BLOCK_OMEGA else "levels_gamma"]
            assert nl == len(H.levels)
            for lvl, lv in enumerate(H.levels):
                Ah = _csr(h, block, lvl, L.MDP_MAT_A)
                scale = abs(lv.A).max()
                assert Ah.shape == lv.A.shape
                assert abs(Ah - lv.A).max() <= 1e-12 * scale
                if lvl + 1 < len(H.levels):
                    agg = L.mdp_level_aggregates(h, block, lvl)
                    assert np.array_equal(agg, lv.agg)
                    P = _csr(h, block, lvl, L.MDP_MAT_P)
                    R = _csr(h, block, lvl, L.MDP_MAT_R)
                    assert abs(P - lv.P).max() <= 1e-13
                    assert (R != P.T).nnz == 0
    finally:
        L.mdp_destroy(h)


def test_interleaved_unknowns_give_the_same_hierarchy():
    """The library orders unknowns as [Omega; Gamma] keeping the caller's
    relative order inside each block, so interleaving fracture unknowns
    among host unknowns must not change anything."""
    sc = synth.tiny_2d(10, seed=1)
    A, b, part = tpfa.assemble(sc)
    # random riffle: positions of the two blocks are mixed, each block's own
    # order is kept
    key = np.where(part == 0, np.arange(A.shape[0]), 0).astype(float)
    key[part == 1] = np.sort(np.random.default_rng(3).uniform(0, part.size - part.sum(), part.sum()))
    perm = np.argsort(key, kind="stable")
    h0 = _host_handle(A, part)
    h1 = _host_handle(A[perm][:, perm].tocsr(), part[perm])
    try:
        for lvl in range(L.mdp_info(h0)["levels_omega"]):
            A0 = _csr(h0, 0, lvl, L.MDP_MAT_A)
            A1 = _csr(h1, 0, lvl, L.MDP_MAT_A)
            assert abs(A0 - A1).max() == 0.0
    finally:
        L.mdp_destroy(h0)
        L.mdp_destroy(h1)


def _expect(code, A, part, **kw):
    with pytest.raises(L.MdpError) as e:
        _host_handle(A, part, **kw)
    assert e.value.code == code, str(e.value)


def test_input_validation_errors():
    sc = synth.tiny_2d(6)
    A, b, part = tpfa.assemble(sc)
    n = A.shape[0]
    # malformed CSR: non-monotone row_ptr, column out of range, bad part
    ptr = A.indptr.copy()
    ptr[3], ptr[4] = ptr[4], ptr[3]
    _expect(L.MDP_EINVAL, (ptr, A.indices, A.data), part)
    col = A.indices.copy()
    col[5] = n + 3
    _expect(L.MDP_EINVAL, (A.indptr, col, A.data), part)
    bad = part.copy()
    bad[0] = 2
    _expect(L.MDP_EINVAL, A, bad)
    # NaN in the values
    val = A.data.copy()
    val[7] = np.nan
    _expect(L.MDP_ENAN, (A.indptr, A.indices, val), part)
    # zero and negative diagonal
    D = A.tolil()
    D[2, 2] = 0.0
    _expect(L.MDP_ENONPOS_DIAG, D.tocsr(), part)
    D[2, 2] = -1.0
    _expect(L.MDP_ENONPOS_DIAG, D.tocsr(), part)
    # bad options
    _expect(L.MDP_EINVAL, A, part, restart=65)
    _expect(L.MDP_EINVAL, A, part, precision=7)
    _expect(L.MDP_EINVAL, A, part, rtol=0.0)
    _expect(L.MDP_EINVAL, A, part, pre_sweeps=0)
    _expect(L.MDP_EINVAL, A, part, post_sweeps=9)


def test_singular_system_is_reported():
    """Pure-Neumann host (no Dirichlet boundary): A 1 = 0, so the coarsest
    level of the S~ hierarchy is singular."""
    sc = synth.tiny_2d(8)
    sc = synth.Scenario(2, sc.n, sc.k_host, sc.fractures, {})
    A, b, part = tpfa.assemble(sc)
    assert np.allclose(A @ np.ones(A.shape[0]), 0.0, atol=1e-12)
    _expect(L.MDP_ESINGULAR, A, part)


def test_singular_nonsymmetric_system_is_reported():
    """The same pure-Neumann system with its rows scaled by positive factors
    (nonsymmetric, A_OG != A_GO^T): still A 1 = 0, still rejected.  With a
    Dirichlet boundary the row-scaled system is accepted."""
    sc0 = synth.tiny_2d(8)
    sc = synth.Scenario(2, sc0.n, sc0.k_host, sc0.fractures, {})
    A, b, part = tpfa.assemble(sc)
    rs = 1.0 + 3.0 * synth.random_vector(A.shape[0], 2) ** 2
    As = sp.csr_matrix(sp.diags(rs) @ A)
    assert abs(As - As.T).max() > 0
    _expect(L.MDP_ESINGULAR, As, part)
    A2, b2, part2 = tpfa.assemble(sc0)
    h = _host_handle(sp.csr_matrix(sp.diags(rs) @ A2), part2)
    L.mdp_destroy(h)


def test_singular_part_of_a_grounded_system_is_reported():
    """Directed coupling: rows 0..k-1 (zero row sums) reference only each
    other, while the rest is grounded and references them.  Row-wise the
    first block cannot reach a Dirichlet row, so A is singular although the
    whole graph is connected."""
    n, k = 6, 3
    A = np.zeros((n, n))
    for i in range(k):  # closed, zero-row-sum block (a directed ring)
        A[i, i] = 1.0
        A[i, (i + 1) % k] = -1.0
    for i in range(k, n):  # grounded rows that also couple to the block
        A[i, i] = 3.0
        A[i, i - 1] = -1.0
    part = np.zeros(n, dtype=np.int32)
    assert abs(np.linalg.det(A)) < 1e-12
    _expect(L.MDP_ESINGULAR, sp.csr_matrix(A), part)


def test_no_fracture_unknowns_allowed():
    n = 12
    sc = synth.Scenario(2, n, np.ones(n * n), [], {(0, 0): 1.0, (0, 1): 0.0})
    A, b, part = tpfa.assemble(sc)
    h = _host_handle(A, part)
    try:
        info = L.mdp_info(h)
        assert info["n_gamma"] == 0 and info["levels_gamma"] == 0
    finally:
        L.mdp_destroy(h)


def test_host_only_handle_refuses_solve():
    import ctypes
    sc = synth.tiny_2d(6)
    A, b, part = tpfa.assemble(sc)
    h = _host_handle(A, part)
    try:
        rc = L.lib.mdp_solve(h, ctypes.c_void_p(8), ctypes.c_void_p(8), 1, A.shape[0], None, None)
        assert rc == L.MDP_EINVAL
    finally:
        L.mdp_destroy(h)


def test_server_lifecycle_without_device_work():
    """A server starts and stops its slots with no request; bad slot counts
    and host-only handles are refused (no device call is made)."""
    import ctypes
    out = ctypes.c_void_p()
    assert L.lib.mdp_server_create(0, 0, ctypes.byref(out)) == L.MDP_EINVAL
    assert L.lib.mdp_server_create(0, 65, ctypes.byref(out)) == L.MDP_EINVAL
    srv = L.mdp_server_create(1 << 20, 3)
    sc = synth.tiny_2d(6)
    A, b, part = tpfa.assemble(sc)
    h = _host_handle(A, part)
    try:
        assert L.lib.mdp_server_register(srv, h) == L.MDP_EINVAL
        t = ctypes.c_uint64()
        assert L.lib.mdp_submit(srv, h, ctypes.c_void_p(8), ctypes.c_void_p(8), 1, ctypes.byref(t)) == L.MDP_EINVAL
        assert L.lib.mdp_poll(srv, 1, None) == L.MDP_EINVAL
        L.mdp_server_set_grouping(srv, False)
        L.mdp_server_set_grouping(srv, True)
        assert L.lib.mdp_server_set_grouping(srv, 2) == L.MDP_EINVAL
        assert L.lib.mdp_server_set_grouping(None, 1) == L.MDP_EINVAL
        assert L.mdp_server_counts(srv) == {"columns": 0, "grouped": 0}
        assert L.lib.mdp_server_counts(None, None, None) == L.MDP_EINVAL
    finally:
        L.mdp_destroy(h)
        L.mdp_server_destroy(srv)


def test_unknown_block_form_rejected():
    sc = synth.tiny_2d(6)
    A, b, part = tpfa.assemble(sc)
    o = L.mdp_options_default(flags=L.MDP_HOST_ONLY, block_form=7)
    with pytest.raises(L.MdpError) as e:
        L.mdp_setup(A, part, o)
    assert e.value.code == L.MDP_EINVAL


def test_unknown_flag_bits_rejected():
    sc = synth.tiny_2d(6)
    A, b, part = tpfa.assemble(sc)
    o = L.mdp_options_default(flags=L.MDP_HOST_ONLY | 64)
    with pytest.raises(L.MdpError) as e:
        L.mdp_setup(A, part, o)
    assert e.value.code == L.MDP_EINVAL


def _all_levels(h):
    info = L.mdp_info(h)
    out = []
    for block, nl in ((0, info["levels_omega"]), (1, info["levels_gamma"])):
        for lvl in range(nl):
            for mat in (L.MDP_MAT_A, L.MDP_MAT_P, L.MDP_MAT_R):
                try:
                    out.append(L.mdp_level_export(h, block, lvl, mat))
                except L.MdpError:
                    out.append(None)
            if lvl + 1 < nl:
                out.append(L.mdp_level_aggregates(h, block, lvl))
    return info, out


def test_hierarchy_file_round_trip(tmp_path):
    """mdp_save / mdp_load reproduce the whole host setup bit for bit."""
    sc = synth.regular_3d(n=10, k_par=1e4, kappa=1e-4, seed=3)
    A, b, part = tpfa.assemble(sc)
    h = _host_handle(A, part, max_coarse=30)
    path = str(tmp_path / "h.mdph")
    try:
        L.mdp_save(h, path)
        o = L.mdp_options_default(flags=L.MDP_HOST_ONLY, max_coarse=30, precision=L.MDP_MIXED)
        h2 = L.mdp_load(path, o)
        try:
            i1, l1 = _all_levels(h)
            i2, l2 = _all_levels(h2)
            assert i1 == i2 and i1["levels_omega"] >= 2
            for a, c in zip(l1, l2):
                if a is None or c is None:
                    assert a is None and c is None
                elif isinstance(a, tuple):
                    assert all(np.array_equal(x, y) for x, y in zip(a[:3], c[:3])) and a[3] == c[3]
                else:
                    assert np.array_equal(a, c)
        finally:
            L.mdp_destroy(h2)
        # AMG options must match the file's
        with pytest.raises(L.MdpError) as e:
            L.mdp_load(path, L.mdp_options_default(flags=L.MDP_HOST_ONLY, max_coarse=31))
        assert e.value.code == L.MDP_EINVAL
    finally:
        L.mdp_destroy(h)


def test_hierarchy_file_version_1_still_read(tmp_path):
    """A file of the first format version (no fused restrictions) loads and
    gives the same hierarchy; its V-cycles restrict the residual instead."""
    sc = synth.regular_3d(n=10, k_par=1e4, kappa=1e-4, seed=3)
    A, b, part = tpfa.assemble(sc)
    h = _host_handle(A, part, max_coarse=30)
    path = tmp_path / "h.mdph"
    try:
        L.mdp_save(h, str(path))
        old = tmp_path / "h1.mdph"
        old.write_bytes(to_version_1(path.read_bytes()))
        h1 = L.mdp_load(str(old), L.mdp_options_default(flags=L.MDP_HOST_ONLY, max_coarse=30))
        try:
            i0, l0 = _all_levels(h)
            i1, l1 = _all_levels(h1)
            assert i0 == i1
            for a, c in zip(l0, l1):
                if isinstance(a, tuple):
                    assert all(np.array_equal(x, y) for x, y in zip(a[:3], c[:3])) and a[3] == c[3]
                elif a is not None:
                    assert np.array_equal(a, c)
        finally:
            L.mdp_destroy(h1)
    finally:
        L.mdp_destroy(h)


def test_hierarchy_file_rejects_damage(tmp_path):
    sc = synth.tiny_2d(9, seed=2)
    A, b, part = tpfa.assemble(sc)
    h = _host_handle(A, part)
    path = tmp_path / "h.mdph"
    try:
        L.mdp_save(h, str(path))
    finally:
        L.mdp_destroy(h)
    data = path.read_bytes()
    o = L.mdp_options_default(flags=L.MDP_HOST_ONLY)
    cases = {"truncated": data[: len(data) // 2], "empty": b"", "flipped": bytearray(data),
             "tag": b"XXXXXXXX" + data[8:]}
    cases["flipped"][len(data) // 3] ^= 0x40
    for name, blob in cases.items():
        p = tmp_path / f"bad_{name}"
        p.write_bytes(bytes(blob))
        with pytest.raises(L.MdpError) as e:
            L.mdp_load(str(p), o)
        assert e.value.code == L.MDP_EINVAL, name
    with pytest.raises(L.MdpError):
        L.mdp_load(str(tmp_path / "missing"), o)
    # a consistent checksum over inconsistent contents: n changed (the field
    # after the tag, version and AMG options) and the checksum recomputed
    def fnv(b):
        h = 1469598103934665603
        for c in b:
            h = ((h ^ c) * 1099511628211) & (2 ** 64 - 1)
        return h
    body = bytearray(data[:-8])
    off = 8 + 4 + 8 + 3 * 4
    body[off:off + 4] = (int.from_bytes(body[off:off + 4], "little") + 1).to_bytes(4, "little")
    p = tmp_path / "bad_sizes"
    p.write_bytes(bytes(body) + fnv(bytes(body)).to_bytes(8, "little"))
    with pytest.raises(L.MdpError) as e:
        L.mdp_load(str(p), o)
    assert e.value.code == L.MDP_EINVAL and "not a valid" in str(e.value)
    good = tmp_path / "good"
    good.write_bytes(data[:-8] + fnv(data[:-8]).to_bytes(8, "little"))
    L.mdp_destroy(L.mdp_load(str(good), o))  # the checksum is FNV-1a 64 over the body


def test_noalloc_apply_refuses_operators_beyond_its_scratch():
    """mdp_apply_noalloc stages mixed-precision operators in a fixed 64 MiB
    array: at most 8,388,608 unknowns.  A host-only handle of 8,410,000
    unknowns is refused for its size before anything touches a device."""
    import ctypes
    n = 2900
    sc = synth.Scenario(2, n, np.ones(n * n), [], {(0, 0): 1.0, (0, 1): 0.0})
    A, b, part = tpfa.assemble(sc)
    h = _host_handle(A, part, precision=L.MDP_MIXED)
    try:
        rc = L.lib.mdp_apply_noalloc(h, L.MDP_OP_ML, ctypes.c_void_p(8), ctypes.c_void_p(8), None)
        assert rc == L.MDP_EINVAL and "exceeds the no-allocation limit of 8388608" in L.mdp_last_error()
        rc = L.lib.mdp_apply_noalloc(h, L.MDP_OP_A, ctypes.c_void_p(8), ctypes.c_void_p(8), None)
        assert rc == L.MDP_EINVAL and "host-only" in L.mdp_last_error()
    finally:
        L.mdp_destroy(h)


def test_tune_file_errors(tmp_path):
    """A tuning file that cannot be created is refused; an unreadable line
    is skipped; NULL stops recording."""
    with pytest.raises(L.MdpError) as e:
        L.mdp_tune_file(str(tmp_path / "no" / "such" / "dir" / "t.txt"))
    assert e.value.code == L.MDP_EINVAL
    p = tmp_path / "t.txt"
    p.write_text("8 10 10 3 28 64  1 0 0 0 8 4\ngarbage\n8 10 10 3 28 64  1 1 0 0 8 4\n")
    L.mdp_tune_file(str(p))
    L.mdp_tune_file(None)


def test_binding_constants_match_the_header():
    """Every integer constant the C header defines has the same value in the
    Python binding (status codes, flags, forms, operators, blocks)."""
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "mdp.h")).read()
    seen = 0
    for name, val in re.findall(r"^#define (MDP_[A-Z0-9_]+) \(?(-?\d+)u?\)?", hdr, re.M):
        if hasattr(L, name):
            assert getattr(L, name) == int(val), name
            seen += 1
    for name in ("MDP_STAGNATED", "MDP_FALLBACK_FP64", "MDP_GRAPHS", "MDP_ENAN", "MDP_SMOOTH_GS",
                 "MDP_HOST_PRODUCTS"):
        assert hasattr(L, name), name
    assert seen >= 30


def test_fallback_flag_accepted_and_stats_field_present():
    sc = synth.tiny_2d(6)
    A, b, part = tpfa.assemble(sc)
    o = L.mdp_options_default(precision=L.MDP_MIXED, flags=L.MDP_HOST_ONLY | L.MDP_FALLBACK_FP64)
    h = L.mdp_setup(A, part, o)
    L.mdp_destroy(h)
    assert "fallback" in L.mdp_stats().as_dict()
    o = L.mdp_options_default(flags=L.MDP_HOST_ONLY | L.MDP_HOST_PRODUCTS)
    L.mdp_destroy(L.mdp_setup(A, part, o))
    o = L.mdp_options_default(flags=L.MDP_HOST_ONLY | 64)
    with pytest.raises(L.MdpError) as e:
        L.mdp_setup(A, part, o)
    assert e.value.code == L.MDP_EINVAL


def test_residual_history_of_a_handle_without_solves():
    import ctypes
    sc = synth.tiny_2d(6)
    A, b, part = tpfa.assemble(sc)
    h = L.mdp_setup(A, part, L.mdp_options_default(flags=L.MDP_HOST_ONLY))
    try:
        assert len(L.mdp_residual_history(h)) == 0
        assert L.lib.mdp_residual_history(h, None, -1, None) == L.MDP_EINVAL
        assert L.lib.mdp_residual_history(h, None, 3, None) == L.MDP_EINVAL
        assert L.lib.mdp_residual_history(None, None, 0, None) == L.MDP_EINVAL
    finally:
        L.mdp_destroy(h)


def test_multi_rhs_memory_of_a_handle_without_a_batch(monkeypatch):
    sc = synth.tiny_2d(6)
    A, b, part = tpfa.assemble(sc)
    h = L.mdp_setup(A, part, L.mdp_options_default(flags=L.MDP_HOST_ONLY))
    try:
        monkeypatch.setenv("MDP_MULTI_RHS_BYTES", "12345")
        m = L.mdp_multi_rhs_memory(h)
        assert m["plan_bytes"] == 0 and m["shared_bytes"] == 0 and m["budget"] == 12345
    finally:
        L.mdp_destroy(h)
    with pytest.raises(L.MdpError):
        L.mdp_multi_rhs_memory(None)
