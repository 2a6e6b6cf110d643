"""Host-side tests of the C ABI (no GPU): symbol exports, input validation, and the
planner's tables (JW Pauli sum, compiled x-groups, excitation signs, pass plan) checked
against the oracle's dense and ladder-operator constructions."""
import re
import os
import ctypes

import numpy as np
import pytest

from oracle import dense, hamiltonian, fermion, ansatz
from paper_2402_17993_amd import inputs, ucc
from paper_2402_17993_amd.inputs import make_integrals, uccsd_excitations

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(not os.path.exists(ucc.LIB_PATH), reason="libucc.so not built")


def host_ctx(n, ne, seed=0, exc=None, **kw):
    h1, h2 = make_integrals(n // 2, seed)
    if exc is None:
        exc = uccsd_excitations(n, ne)
    return ucc.Context(n, ne, h1, h2, exc, host_only=True, **kw), h1, h2, exc


def logical_to_phys(n, ne):
    idx = np.arange(1 << n)
    return (idx >> ne) | ((idx & ((1 << ne) - 1)) << (n - ne))


# ---------------------------------------------------------------- ABI surface

def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "ucc.h")).read()
    declared = set(re.findall(r"\b(ucc_[a-z0-9_]+)\s*\(", header))
    declared -= {"ucc_status"}
    L = ctypes.CDLL(ucc.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(ucc.EXPORTED)


@pytest.mark.parametrize("bad", [
    dict(n=7), dict(n=32), dict(ne=3), dict(ne=8),
    dict(exc=[[0, -1, 1, -1]]),            # occupied -> occupied
    dict(exc=[[0, -1, 5, -1]]),            # spin flip (alpha -> beta)
    dict(exc=[[1, 0, 4, 5]]),              # i > j
    dict(exc=[[0, 1, 4, 5], [0, 1, 4, 5]]),  # duplicate
    dict(h1_asym=True), dict(h2_asym=True), dict(tile_qubits=20), dict(block_threads=300),
    dict(block_threads_rev=128), dict(block_threads_exp=768), dict(autotune=True),
    dict(store_states=3), dict(store_states=1, tile_qubits=14), dict(trotter_steps=65),
    dict(trotter_steps=-1), dict(trotter_order=3),
    dict(store_states=1, tile_qubits=7, tile_qubits_rev=6),
    dict(tile_qubits_rev=15), dict(store_states=1, tile_qubits_rev=14),
])
def test_invalid_inputs_are_rejected(bad):
    n, ne = bad.get("n", 8), bad.get("ne", 4)
    h1, h2 = make_integrals(4, 0)
    if bad.get("h1_asym"):
        h1 = h1.copy()
        h1[0, 1] += 1e-6
    if bad.get("h2_asym"):
        h2 = h2.copy()
        h2[0, 1, 2, 3] += 1e-6
    exc = np.array(bad.get("exc", uccsd_excitations(8, 4)), dtype=np.int32)
    kw = {k: bad[k] for k in ("tile_qubits", "tile_qubits_rev", "block_threads",
                              "block_threads_rev", "block_threads_exp", "autotune",
                              "store_states", "trotter_steps", "trotter_order") if k in bad}
    with pytest.raises(ucc.UCCError) as ei:
        ucc.Context(n, ne, h1[: n // 2, : n // 2] if n <= 8 else np.zeros((n // 2,) * 2),
                    h2 if n == 8 else np.zeros((n // 2,) * 4), exc, host_only=True, **kw)
    assert ei.value.status == -1


def test_host_only_context_refuses_evaluation():
    ctx, *_ = host_ctx(8, 4)
    with pytest.raises(ucc.UCCError):
        ctx.energy(np.zeros(ctx.n_exc))


# ---------------------------------------------------------------- JW Pauli sum

@pytest.mark.parametrize("ns,ne,seed", [(3, 2, 1), (4, 4, 0)])
def test_pauli_sum_reconstructs_dense_hamiltonian(ns, ne, seed):
    n = 2 * ns
    ctx, h1, h2, _ = host_ctx(n, ne, seed)
    x, z, c = ctx.pauli_terms()
    H = np.zeros((1 << n, 1 << n), dtype=complex)
    for xi, zi, ci in zip(x, z, c):
        lab = "".join("I" if not (xi >> q) & 1 and not (zi >> q) & 1 else
                      "X" if (xi >> q) & 1 and not (zi >> q) & 1 else
                      "Y" if (xi >> q) & 1 else "Z" for q in range(n))
        H += ci * dense.pauli_matrix(lab)
    h, g = hamiltonian.spin_orbital_integrals(h1, h2)
    np.testing.assert_allclose(H, dense.hamiltonian_dense(h, g), atol=1e-12)


def test_pauli_string_counts():
    # counts quoted for the workloads (8 / 12 / 16 qubits)
    for n, ne, strings, groups in [(8, 4, 361, 51), (12, 8, 1819, 286), (16, 8, 5793, 981)]:
        ctx, *_ = host_ctx(n, ne)
        info = ctx.plan_info()
        assert info["n_pauli"] == strings
        assert info["n_groups"] == groups


# ---------------------------------------------------------------- compiled groups

@pytest.mark.parametrize("ns,ne,seed", [(4, 4, 0), (5, 6, 2), (5, 4, 3)])
def test_group_table_reproduces_hamiltonian_in_sector(ns, ne, seed):
    n = 2 * ns
    ctx, h1, h2, _ = host_ctx(n, ne, seed)
    tab = ctx.group_table()
    perm = np.array(ctx.plan_info()["perm"])
    h, g = hamiltonian.spin_orbital_integrals(h1, h2)
    N = 1 << n
    l2p = logical_to_phys(n, ne)
    # physical matrix Hp[P(a), P(b)] = <a|H|b>, columns b in the N / S_z sector, from the
    # oracle's ladder-operator H (pinned to the dense Kronecker H in the oracle tests)
    lv = np.arange(N)
    lsec = (np.bitwise_count(lv & 0x5555_5555) == ne // 2) & (np.bitwise_count(lv & 0xAAAA_AAAA) == ne // 2)
    Hp = np.zeros((N, N))
    for b in np.flatnonzero(lsec):
        e = np.zeros(N, dtype=complex)
        e[b] = 1.0
        Hp[l2p, l2p[b]] = hamiltonian.apply_h(h, g, e).real
    v = np.arange(N)
    occ = ((v[:, None] >> np.arange(n)) & 1).astype(float)
    Hc = np.zeros((N, N))
    diag = tab["c0"] + occ @ tab["a"] + np.einsum("vr,rs,vs->v", occ, np.triu(tab["b"], 1), occ)
    Hc[v, v] += diag
    for gi in range(1, len(tab["x"])):
        x = int(tab["x"][gi])
        pos = [q for q in range(n) if (x >> q) & 1]
        P = sum(((v >> p) & 1) << j for j, p in enumerate(pos))
        ok = (tab["valid"][gi] >> P) & 1 == 1
        val = tab["A"][gi][P] + np.einsum("vr,vr->v", occ, tab["B"][gi][P])
        sgn = np.where(np.bitwise_count(v & int(tab["m"][gi])) & 1, -1.0, 1.0)
        vv = v[ok]
        Hc[vv ^ x, vv] += (sgn * val)[ok]
    amask = sum(1 << int(perm[q]) for q in range(0, n, 2))
    bmask = sum(1 << int(perm[q]) for q in range(1, n, 2))
    sec = (np.bitwise_count(v & amask) == ne // 2) & (np.bitwise_count(v & bmask) == ne // 2)
    S = np.flatnonzero(sec)
    np.testing.assert_allclose(Hc[np.ix_(S, S)], Hp[np.ix_(S, S)], atol=1e-12)
    # nothing leaves the sector
    assert np.max(np.abs(Hc[np.ix_(~sec, S)])) == 0.0


# ---------------------------------------------------------------- excitation signs

@pytest.mark.parametrize("n,ne", [(8, 4), (10, 6), (12, 4)])
def test_excitation_signs_match_ladder_operators(n, ne):
    ctx, _, _, exc = host_ctx(n, ne)
    t = ctx.excitation_table()
    l2p = logical_to_phys(n, ne)
    for k, row in enumerate(exc):
        src, dst, s = ansatz.excitation_pairs(n, row)
        up, vp = l2p[src], l2p[dst]
        assert np.all((up & int(t["supp"][k])) == int(t["frm"][k]))
        assert np.all((up ^ vp) == int(t["supp"][k]))
        pred = t["sigma"][k] * np.where(np.bitwise_count(up & int(t["m"][k])) & 1, -1, 1)
        assert np.array_equal(pred, s)


# ---------------------------------------------------------------- pass plan

@pytest.mark.parametrize("n,ne,kf,ke,kr,ss,stored", [
    (8, 4, 0, 0, 0, 0, 1), (12, 8, 8, 9, 7, 0, 0), (16, 8, 0, 0, 0, 0, 1), (16, 8, 0, 0, 0, 2, 0),
    (18, 10, 0, 0, 0, 0, 1), (18, 10, 10, 11, 9, 0, 0), (18, 10, 14, 12, 13, 0, 0),
    (18, 10, 0, 12, 11, 1, 1), (18, 10, 0, 0, 0, 2, 0), (18, 10, 14, 14, 14, 2, 0)])
def test_pass_plan_covers_everything_in_order(n, ne, kf, ke, kr, ss, stored):
    ctx, _, _, exc = host_ctx(n, ne, tile_qubits=kf, tile_qubits_exp=ke, tile_qubits_rev=kr,
                              store_states=ss)
    info = ctx.plan_info()
    assert info["store_states"] == stored
    passes = ctx.pass_table()
    et = ctx.excitation_table()
    gt = ctx.group_table()
    fwd = [p for p in passes if p["kind"] == 0]
    exp_ = [p for p in passes if p["kind"] == 1]
    rev = [p for p in passes if p["kind"] == 2]
    assert len(fwd) == info["n_fwd_passes"] and len(exp_) == info["n_exp_passes"]
    K = len(exc)
    assert np.array_equal(np.concatenate([p["items"] for p in fwd]), np.arange(K))
    assert np.array_equal(np.concatenate([p["items"] for p in rev]), np.arange(K)[::-1])
    check_commuting_reorder(np.concatenate([p["items"] for p in fwd]), np.arange(K), et["supp"])
    for group, k, c0 in ((fwd, info["tile_qubits"], info["contiguous_fwd"]),
                         (rev, info["tile_qubits_rev"], info["contiguous_rev"])):
        for p in group:
            assert bin(p["local"]).count("1") == k
            assert p["local"] & ((1 << c0) - 1) == (1 << c0) - 1
            for e in p["items"]:
                assert int(et["supp"][e]) & ~p["local"] == 0
    if stored:  # the reverse passes are the forward windows in mirror order
        assert info["tile_qubits"] == info["tile_qubits_rev"] and len(rev) == len(fwd)
        for r, f in zip(rev, fwd[::-1]):
            assert r["local"] == f["local"]
            assert np.array_equal(r["items"], np.asarray(f["items"])[::-1])
    seen = np.concatenate([p["items"] for p in exp_])
    assert np.array_equal(np.sort(seen), np.arange(info["n_groups"]))
    for p in exp_:
        assert bin(p["local"]).count("1") == info["tile_qubits_exp"]
        for gi in p["items"]:
            assert int(gt["x"][gi]) & ~p["local"] == 0


def check_commuting_reorder(applied, listed, supp):
    """applied is a permutation of listed in which every pair of factors whose order changed
    acts on disjoint spin orbitals (so the product is unchanged)."""
    applied, listed = np.asarray(applied), np.asarray(listed)
    assert np.array_equal(np.sort(applied), np.sort(listed))
    pos = {int(e): i for i, e in enumerate(applied)}
    for x in range(len(listed)):
        for y in range(x + 1, len(listed)):
            a, b = int(listed[x]), int(listed[y])
            if pos[a] > pos[b]:
                assert int(supp[a]) & int(supp[b]) == 0, (a, b)


@pytest.mark.parametrize("n,ne,kw", [(12, 8, dict(tile_qubits=8, tile_qubits_rev=8)),
                                     (16, 8, dict(store_states=2)), (16, 8, dict(store_states=1))])
def test_windows_of_a_magnitude_ordered_list(n, ne, kw):
    # a scattered Trotter order: windows may take later factors ahead of earlier ones they
    # commute with; the applied sequence is then a commuting rearrangement of the list
    h1, h2 = make_integrals(n // 2, 0)
    exc = uccsd_excitations(n, ne)
    exc = exc[inputs.magnitude_order(h1, h2, ne, exc)]
    ctx = ucc.Context(n, ne, h1, h2, exc, host_only=True, **kw)
    passes = ctx.pass_table()
    et = ctx.excitation_table()
    fwd = np.concatenate([p["items"] for p in passes if p["kind"] == 0])
    rev = np.concatenate([p["items"] for p in passes if p["kind"] == 2])
    K = len(exc)
    assert not np.array_equal(fwd, np.arange(K))  # something was moved
    check_commuting_reorder(fwd, np.arange(K), et["supp"])
    check_commuting_reorder(rev, np.arange(K)[::-1], et["supp"])
    if ctx.plan_info()["store_states"]:
        assert np.array_equal(rev, fwd[::-1])


# ---------------------------------------------------------------- serving (host side)

def test_batch_compatibility_and_job_footprint():
    exc = uccsd_excitations(12, 8)
    a = ucc.Context(12, 8, *make_integrals(6, 1), exc, host_only=True)
    b = ucc.Context(12, 8, *make_integrals(6, 2), exc, host_only=True)
    assert a.batch_compatible(b) and b.batch_compatible(a) and a.batch_compatible(a)
    # another size, another excitation list, another tiling: separate batches
    c = ucc.Context(16, 8, *make_integrals(8, 1), uccsd_excitations(16, 8), host_only=True)
    d = ucc.Context(12, 8, *make_integrals(6, 2), exc[:-1], host_only=True)
    e = ucc.Context(12, 8, *make_integrals(6, 2), exc, host_only=True, tile_qubits=10)
    f = ucc.Context(12, 8, *make_integrals(6, 2), exc, host_only=True, store_states=2)
    assert not a.batch_compatible(c) and not a.batch_compatible(d) and not a.batch_compatible(e)
    assert not a.batch_compatible(f)
    # footprint: two complex128 vectors plus partial sums, rows and one table row
    info = a.plan_info()
    S = 16 << 12
    assert 2 * S < info["job_footprint"] < 2 * S + (1 << 20)
    # stored states: one more vector per forward pass but the last
    info = c.plan_info()
    S = 16 << 16
    assert info["store_states"] == 1
    extra = (info["n_fwd_passes"] - 1) * S
    assert 2 * S + extra < info["job_footprint"] < 2 * S + extra + (4 << 20)


def test_server_argument_errors():
    with pytest.raises(ucc.UCCError) as ei:
        ucc.Server(slots=0)
    assert ei.value.status == -1
    with pytest.raises(ucc.UCCError) as ei:
        ucc.Server(slots=8, max_queue=-1)
    assert ei.value.status == -1
    L = ucc.lib()
    t = ucc.ctypes.c_uint64()
    assert L.ucc_submit(None, None, None, 1, 0.1, 0, ucc.ctypes.byref(t)) == -1
    done = ucc.ctypes.c_int32()
    assert L.ucc_poll(None, 1, ucc.ctypes.byref(done), None, None, None) == -1
    assert L.ucc_cancel(None, 1) == -1
    L.ucc_server_destroy(None)  # accepted


def test_launch_mode_resolution():
    # one-tile states take the whole-evaluation launch by default; larger ones cannot
    for n, ne, want in ((4, 2, 2), (8, 4, 2), (12, 8, 2), (16, 8, 1)):
        ctx, *_ = host_ctx(n, ne)
        assert ctx.plan_info()["launch_mode"] == want, (n, want)
    ctx, *_ = host_ctx(12, 8, launch_mode=1)
    assert ctx.plan_info()["launch_mode"] == 1
    with pytest.raises(ucc.UCCError) as ei:
        host_ctx(16, 8, launch_mode=2)
    assert ei.value.status == -1
    with pytest.raises(ucc.UCCError):  # a 12-qubit state split into tiles is not one tile
        host_ctx(12, 8, launch_mode=2, tile_qubits=8)


@pytest.mark.parametrize("n,ne,M,order,kw", [(8, 4, 3, 1, {}), (12, 8, 2, 2, {}),
                                             (16, 8, 2, 2, {}), (16, 8, 3, 1, dict(store_states=2))])
def test_trotter_product_plan(n, ne, M, order, kw):
    # the factors of Eq. 5 (M slices) or Eq. 6 (list, then reversed list, per slice) in order,
    # every forward pass a window of consecutive factors, the reverse passes in the opposite order
    ctx, _, _, exc = host_ctx(n, ne, trotter_steps=M, trotter_order=order, **kw)
    info = ctx.plan_info()
    assert (info["trotter_steps"], info["trotter_order"]) == (M, order)
    K = len(exc)
    L = K * M * order
    passes = ctx.pass_table()
    fwd = np.concatenate([p["items"] for p in passes if p["kind"] == 0])
    rev = np.concatenate([p["items"] for p in passes if p["kind"] == 2])
    assert np.array_equal(fwd, np.arange(L)) and np.array_equal(rev, np.arange(L)[::-1])
    et = ctx.excitation_table()
    one = list(range(K)) + (list(range(K - 1, -1, -1)) if order == 2 else [])
    seq = np.array(one * M)
    for p in passes:
        if p["kind"] != 1:
            for o in p["items"]:
                assert int(et["supp"][seq[o]]) & ~p["local"] == 0


# ---------------------------------------------------------------- Trotter-free generator plan

@pytest.mark.parametrize("n,ne,kw", [(8, 4, {}), (12, 8, dict(tile_qubits_exp=8)),
                                     (16, 8, {}), (18, 10, dict(tile_qubits_exp=12))])
def test_generator_plan_covers_every_excitation_once(n, ne, kw):
    ctx, _, _, exc = host_ctx(n, ne, **kw)
    local, where = ctx.generator_passes()
    info = ctx.plan_info()
    t = ctx.excitation_table()
    k = min(n, kw.get("tile_qubits_exp", 14))
    assert len(local) >= 1 and np.all(where >= 0) and np.all(where < len(local))
    for m in local:
        assert bin(int(m)).count("1") == k
    # each excitation's support lies inside its pass's local qubits
    for e, p in enumerate(where):
        assert int(t["supp"][e]) & ~int(local[p]) == 0
    # the generator needs no more passes than the Hamiltonian's expectation sweep (its
    # supports are x-masks of H's groups) plus the LDS splits
    assert len(local) <= info["n_exp_passes"] + 2
    ctx.close()


@pytest.mark.parametrize("n,ne,kw", [(8, 4, {}), (12, 8, dict(tile_qubits=8, tile_qubits_rev=8)),
                                     (12, 4, dict(store_states=2, tile_qubits_rev=9)),
                                     (16, 8, dict(trotter_steps=2)), (18, 10, {})])
def test_partials_windows_hold_every_factor_once(n, ne, kw):
    # the Trotter-free gradient's partials-only reverse passes: order-free windows of the
    # reverse tile, every factor of the product in exactly one, inside its local qubits
    ctx, _, _, exc = host_ctx(n, ne, **kw)
    local, where = ctx.partials_passes()
    info = ctx.plan_info()
    t = ctx.excitation_table()
    L = len(exc) * info["trotter_steps"] * info["trotter_order"]
    assert len(where) == L and np.all(where >= 0) and np.all(where < len(local))
    for m in local:
        assert bin(int(m)).count("1") == info["tile_qubits_rev"]
    for o, w in enumerate(where):
        assert int(t["supp"][o % len(exc)]) & ~int(local[w]) == 0
    # never more windows than the Trotter-ordered reverse sweep
    assert 1 <= len(local) <= info["n_rev_passes"]
    if (n, ne) == (18, 10):
        assert len(local) < info["n_rev_passes"]
    ctx.close()


# ---------------------------------------------------------------- FMO two-body energy (Eq. 1)

def test_fmo2_energy_assembly():
    r = np.random.default_rng(3)
    for nf in (2, 3, 5):
        em = r.normal(size=nf)
        pairs = [(i, j) for i in range(nf) for j in range(i)]
        ed = r.normal(size=len(pairs))
        # Eq. 1 as printed, and its equivalent monomer-plus-pair-correction form
        ref = ed.sum() - (nf - 2) * em.sum()
        alt = em.sum() + sum(ed[k] - em[i] - em[j] for k, (i, j) in enumerate(pairs))
        assert abs(ucc.fmo2_energy(em, ed) - ref) < 1e-12 and abs(ref - alt) < 1e-12
    # non-interacting fragments whose pair energies are exactly additive give the monomer sum
    em = np.array([-1.25, -2.5, -0.75])
    ed = np.array([em[1] + em[0], em[2] + em[0], em[2] + em[1]])
    assert ucc.fmo2_energy(em, ed) == em.sum()
    with pytest.raises(ValueError):
        ucc.fmo2_energy(em, ed[:2])
    with pytest.raises(ucc.UCCError):
        ucc.fmo2_energy(em, np.array([0.0, np.nan, 0.0]))


def test_recomputing_sweep_at_the_forward_tile_size_takes_as_many_windows():
    """26 qubits: with 14 local qubits for both sweeps, the recomputing reverse sweep needs no
    more windows than the forward sweep (one per occupied pair); at 13 it needs 2.5x more."""
    ctx14 = host_ctx(26, 14, tile_qubits=14, tile_qubits_rev=14)[0].plan_info()
    ctx13 = host_ctx(26, 14, tile_qubits=14, tile_qubits_rev=13)[0].plan_info()
    assert ctx14["store_states"] == 0 and ctx14["tile_qubits_rev"] == 14
    assert ctx14["n_rev_passes"] <= ctx14["n_fwd_passes"] == 98
    assert ctx13["n_rev_passes"] > 2 * ctx14["n_rev_passes"]


# ---------------------------------------------------------------- two-qubit tapering

def tapered_maps(ctx, n, ne):
    """Stored index -> logical basis state (tapered orbitals filled with what the stored ones
    lack), and the stored sector mask."""
    info = ctx.plan_info()
    ns_ = info["state_qubits"]
    assert info["taper"] == 1 and ns_ == n - 2
    perm = np.array(info["perm"])
    v = np.arange(1 << ns_)
    L = np.zeros_like(v)
    for q in range(n - 2):
        L |= ((v >> perm[q]) & 1) << q
    la = sum(1 << q for q in range(0, n - 2, 2))
    lb = sum(1 << q for q in range(1, n - 2, 2))
    oa = ne // 2 - np.bitwise_count(L & la).astype(np.int64)
    ob = ne // 2 - np.bitwise_count(L & lb).astype(np.int64)
    sec = (oa >= 0) & (oa <= 1) & (ob >= 0) & (ob <= 1)
    L = L | (np.clip(oa, 0, 1) << (n - 2)) | (np.clip(ob, 0, 1) << (n - 1))
    return v, L, sec, oa, ob


@pytest.mark.parametrize("ns,ne,seed", [(4, 4, 0), (5, 6, 2), (5, 4, 3), (6, 6, 1)])
def test_tapered_group_table_reproduces_hamiltonian(ns, ne, seed):
    """The tapered value tables (occupations of the two tapered orbitals folded into masks,
    signs and occupation rows) give the oracle's <a|H|b> on the sector, entry by entry."""
    n = 2 * ns
    ctx, h1, h2, _ = host_ctx(n, ne, seed, taper=1)
    tab = ctx.group_table()
    h, g = hamiltonian.spin_orbital_integrals(h1, h2)
    v, L, sec, oa, ob = tapered_maps(ctx, n, ne)
    nst = n - 2
    S = np.flatnonzero(sec)
    Hp = np.zeros((1 << nst, 1 << nst))
    pos = {int(L[s]): int(s) for s in S}
    for s in S:
        e = np.zeros(1 << n, dtype=complex)
        e[L[s]] = 1.0
        col = hamiltonian.apply_h(h, g, e).real
        for lo in np.flatnonzero(col):
            Hp[pos[int(lo)], s] = col[lo]  # every image is in the sector
    occ = ((v[:, None] >> np.arange(nst)) & 1).astype(float)
    Hc = np.zeros_like(Hp)
    Hc[v, v] += tab["c0"] + occ @ tab["a"] + np.einsum("vr,rs,vs->v", occ, np.triu(tab["b"], 1), occ)
    vt = v | (np.clip(oa, 0, 1) << nst) | (np.clip(ob, 0, 1) << (nst + 1))
    keep = (1 << nst) - 1
    for gi in range(1, len(tab["x"])):
        xt = int(tab["x"][gi])
        pos_ = [q for q in range(n) if (xt >> q) & 1]
        P = sum(((vt >> p) & 1) << j for j, p in enumerate(pos_))
        ok = sec & ((tab["valid"][gi] >> P) & 1 == 1)
        val = tab["A"][gi][P] + np.einsum("vr,vr->v", occ, tab["B"][gi][P])
        sgn = np.where(np.bitwise_count(v & int(tab["m"][gi])) & 1, -1.0, 1.0)
        vv = v[ok]
        Hc[vv ^ (xt & keep), vv] += (sgn * val)[ok]
    np.testing.assert_allclose(Hc[np.ix_(S, S)], Hp[np.ix_(S, S)], atol=1e-12)


@pytest.mark.parametrize("n,ne", [(8, 4), (10, 6), (12, 4)])
def test_tapered_excitation_signs_match_ladder_operators(n, ne):
    ctx, _, _, exc = host_ctx(n, ne, taper=1)
    t = ctx.excitation_table()
    v, L, sec, _, _ = tapered_maps(ctx, n, ne)
    stored = {int(L[s]): int(s) for s in np.flatnonzero(sec)}
    for k, row in enumerate(exc):
        src, dst, s = ansatz.excitation_pairs(n, row)
        ins = np.array([int(x) in stored for x in src])
        up = np.array([stored[int(x)] for x in src[ins]])
        vp = np.array([stored[int(x)] for x in dst[ins]])
        assert np.all((up & int(t["supp"][k])) == int(t["frm"][k]))
        assert np.all((up ^ vp) == int(t["supp"][k]))
        pred = t["sigma"][k] * np.where(np.bitwise_count(up & int(t["m"][k])) & 1, -1, 1)
        assert np.array_equal(pred, s[ins])


def test_tapered_plan_sizes_and_rejections():
    ctx = host_ctx(18, 10, taper=1)[0]
    info = ctx.plan_info()
    assert info["n_qubits"] == 18 and info["state_qubits"] == 16 and info["taper"] == 1
    assert info["job_footprint"] < host_ctx(18, 10)[0].plan_info()["job_footprint"] / 3
    with pytest.raises(ucc.UCCError):
        host_ctx(6, 2, taper=1)
    with pytest.raises(ucc.UCCError):
        ctx.generator_passes()


@pytest.mark.parametrize("n,ne,kw", [(12, 4, dict(tile_qubits=5, tile_qubits_exp=6, tile_qubits_rev=7,
                                                  store_states=2)),
                                     (16, 8, dict(store_states=2)), (12, 8, dict(tile_qubits=6))])
def test_tapered_windows_keep_non_commuting_factors_in_order(n, ne, kw):
    """Tapered plans: factors that share a tapered orbital act on it although their stored
    supports are disjoint; the windows may exchange only factors on disjoint spin orbitals
    (counted over all n_qubits orbitals), in both sweeps and for a magnitude-ordered list."""
    h1, h2 = make_integrals(n // 2, 0)
    exc = uccsd_excitations(n, ne)
    orb = np.array([sum(1 << int(q) for q in row if q >= 0) for row in exc])
    for order in (np.arange(len(exc)), inputs.magnitude_order(h1, h2, ne, exc)):
        ctx = ucc.Context(n, ne, h1, h2, exc[order], host_only=True, taper=1, **kw)
        passes = ctx.pass_table()
        fwd = np.concatenate([p["items"] for p in passes if p["kind"] == 0])
        rev = np.concatenate([p["items"] for p in passes if p["kind"] == 2])
        K = len(exc)
        check_commuting_reorder(fwd, np.arange(K), orb[order])
        check_commuting_reorder(rev, np.arange(K)[::-1], orb[order])


def test_fusion_depth_caps_the_windows():
    """fuse_depth F: no forward or reverse window holds more than F factors, the windows still
    cover the Trotter product in order, and the option is range-checked."""
    n, ne = 18, 10
    free = host_ctx(n, ne)[0]
    capped, _, _, exc = host_ctx(n, ne, fuse_depth=16)
    assert capped.plan_info()["fuse_depth"] == 16
    counts = [len(p["items"]) for p in capped.pass_table() if p["kind"] != 1]
    assert max(counts) <= 16 < max(len(p["items"]) for p in free.pass_table() if p["kind"] != 1)
    fwd = np.concatenate([p["items"] for p in capped.pass_table() if p["kind"] == 0])
    check_commuting_reorder(fwd, np.arange(len(exc)), capped.excitation_table()["supp"])
    for bad in (-1, 257):
        with pytest.raises(ucc.UCCError):
            host_ctx(8, 4, fuse_depth=bad)


def test_fixed_tuning_takes_grouped_passes_where_the_batch_fills_the_chip():
    """Without the autotuner, 18 qubits with stored states: a batch that gives every CU at
    least two items of grouped entries (four forward, two reverse) takes 1024-thread forward and
    reverse passes (the overlapped, grouped forms); a single vector keeps 512."""
    n, ne = 18, 10
    h1, h2 = make_integrals(n // 2, 0)
    exc = uccsd_excitations(n, ne)
    for batch, want in ((64, (1024, 1024, 1024)), (1, (512, 1024, 512))):
        c = ucc.Context(n, ne, h1, h2, exc, host_only=True, max_batch=batch)
        i = c.plan_info()
        assert i["store_states"] == 1
        assert (i["block_threads_fwd"], i["block_threads_exp"], i["block_threads_rev"]) == want, batch
        c.close()


def test_evaluation_graph_plan_and_rejections():
    """launch_mode 3 (the evaluation graph): 512-thread workgroups and tiles of at most 13 qubits
    for every kind, chosen without the autotuner; what the graph cannot take is refused."""
    for n, ne in ((8, 4), (12, 8), (18, 10), (24, 14)):
        h1, h2 = make_integrals(n // 2, 0)
        c = ucc.Context(n, ne, h1, h2, uccsd_excitations(n, ne), launch_mode=3, host_only=True, max_batch=0)
        i = c.plan_info()
        assert i["launch_mode"] == 3
        assert (i["block_threads_fwd"], i["block_threads_exp"], i["block_threads_rev"]) == (512, 512, 512)
        k = min(n, 13)
        assert (i["tile_qubits"], i["tile_qubits_exp"], i["tile_qubits_rev"]) == (k, k, k)
        assert i["n_fwd_passes"] + i["n_exp_passes"] + i["n_rev_passes"] <= 512
        assert i["graph_grid"] == 0  # no launch yet
        c.close()
    h1, h2 = make_integrals(9, 0)
    exc = uccsd_excitations(18, 10)
    for kw in (dict(taper=1), dict(tile_qubits=14), dict(tile_qubits_exp=14), dict(block_threads=1024),
               dict(block_threads_rev=256), dict(graph_wait_us=-1), dict(launch_mode=4)):
        opts = dict(launch_mode=3, host_only=True)
        opts.update(kw)
        with pytest.raises(ucc.UCCError) as e:
            ucc.Context(18, 10, h1, h2, exc, **opts)
        assert e.value.status == ucc.STATUS_CODES["UCC_EINVAL"], kw
    # autotune needs a device context anyway; with launch_mode 3 it is refused before that
    with pytest.raises(ucc.UCCError) as e:
        ucc.Context(18, 10, h1, h2, exc, launch_mode=3, autotune=True)
    assert "launch_mode 3" in str(e.value)
