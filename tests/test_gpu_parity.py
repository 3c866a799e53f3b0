"""GPU parity: the HIP library against the CPU oracle, element by element.

Everything is integer and exact, so the bar is bit-identity: full Delta_1
and theta arrays against oracle.fast, and heights against the paper's printed
heights and the oracle's stored heights for the seeded workloads.
"""
import json
import os
import sys

import numpy as np
import pytest
import torch

import workloads
from oracle import fast

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def qfs():
    import paper_2502_12428_amd as q
    q.lib()
    assert torch.cuda.is_available(), "no GPU"
    return q


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def delta_inputs(p):
    if p == 3:
        F = np.concatenate([workloads.bernoulli_support(3, 5, 0.7, seed=31), workloads.fermat()[None]])
    elif p == 5:
        F, _ = workloads.config_p5_single(0)
    else:
        F = np.concatenate([workloads.bernoulli_support(7, 1, 0.9, seed=71), workloads.config_p7_single(0, 1)[0]])
    return F


@pytest.mark.parametrize("p", [3, 5, 7])
def test_delta1_full_arrays(qfs, p):
    F = delta_inputs(p)
    say("delta1 p=%d batch=%d" % (p, F.shape[0]))
    g, dl, st = qfs.delta1(dev(F), p)
    g, dl, st = host(g), host(dl), host(st)
    assert np.all(st == 0)
    for i, f in enumerate(F):
        want_g = fast.fpow(f, p, p - 1)
        assert np.array_equal(g[i], want_g), "g differs, surface %d" % i
        want_d = fast.delta1(want_g, p, 4 * (p - 1))
        bad = np.flatnonzero(dl[i] != want_d)
        assert bad.size == 0, "Delta_1 differs at %d of %d positions (first %s), surface %d" % (
            bad.size, want_d.size, bad[:5], i)


def test_delta1_ragged_batch_and_invalid_rows(qfs):
    p = 5
    F = workloads.bernoulli_support(p, 7, 0.5, seed=5)
    F[3, 4] = 9  # >= p: that surface reports QFS_EINVAL
    say("delta1 ragged batch=7 with one invalid row")
    g, dl, st = qfs.delta1(dev(F), p)
    st = host(st)
    assert st[3] == qfs.QFS_EINVAL and np.all(np.delete(st, 3) == 0)
    g, dl = host(g), host(dl)
    for i in (0, 6):
        want_g = fast.fpow(F[i], p, p - 1)
        assert np.array_equal(g[i], want_g)
        assert np.array_equal(dl[i], fast.delta1(want_g, p, 16))


@pytest.mark.parametrize("p,iters", [(3, 1), (3, 4), (5, 1), (5, 3), (7, 1), (7, 2)])
def test_theta_against_oracle(qfs, p, iters):
    d = 4 * (p - 1)
    B = 3
    delta = np.stack([workloads.random_dense(p, qfs.len_delta(p), seed=100 * p + s) for s in range(B)])
    a = np.stack([workloads.random_dense(p, qfs.len_g(p), seed=200 * p + s) for s in range(B)])
    a[1] = 0
    a[1, 7] = 1  # a single monomial
    say("theta p=%d iters=%d" % (p, iters))
    out = host(qfs.theta(dev(delta), dev(a), p, iters))
    for i in range(B):
        want = fast.theta_pow(delta[i], a[i], p, iters)
        assert np.array_equal(out[i], want), "theta differs, surface %d" % i
    assert d > 0


def test_theta_zero_iterations_copies(qfs):
    p = 5
    delta = workloads.random_dense(p, qfs.len_delta(p), seed=1)[None]
    a = workloads.random_dense(p, qfs.len_g(p), seed=2)[None]
    say("theta iters=0")
    assert np.array_equal(host(qfs.theta(dev(delta), dev(a), p, 0)), a)


def paper_rows(p):
    doc = json.load(open(os.path.join(GOLD, "paper_heights.json")))
    rows = [e for e in doc["entries"] if e["p"] == p]
    F = np.array([e["coeffs_b4"] for e in rows], dtype=np.uint8)
    H = np.array([0 if e["height"] == "inf" else e["height"] for e in rows], dtype=np.int32)
    return F, H


@pytest.mark.parametrize("p", [5, 7, 11])
def test_height_paper_tables(qfs, p):
    F, H = paper_rows(p)
    say("height paper table p=%d (%d surfaces)" % (p, len(H)))
    got = host(qfs.height(dev(F), p))
    assert got.tolist() == H.tolist()


def test_height_paper_tables_mixed_batch(qfs):
    Fs, Ps, Hs = [], [], []
    for p in (5, 7, 11):
        F, H = paper_rows(p)
        Fs.append(F)
        Ps.append(np.full(len(H), p, dtype=np.int32))
        Hs.append(H)
    F, P, H = np.concatenate(Fs), np.concatenate(Ps), np.concatenate(Hs)
    perm = np.random.default_rng(0).permutation(len(H))
    say("height paper tables, one mixed batch of %d" % len(H))
    got = host(qfs.height(dev(F[perm]), dev(P[perm]), max_p=11))
    assert got.tolist() == H[perm].tolist()


def load_golden(name):
    path = os.path.join(GOLD, "heights_%s.npz" % name)
    if not os.path.exists(path):
        pytest.skip("golden heights for %s not generated" % name)
    z = np.load(path)
    F, P = workloads.CONFIGS[name]()
    sys.path.insert(0, GOLD)
    from make_golden import input_digest
    assert str(z["sha256"]) == input_digest(F, P), "workload generator changed since the golden file was written"
    return F, P, z["heights"].astype(np.int32)


@pytest.mark.parametrize("name", ["p5_single", "p7_single", "p5_batch8192", "p7_batch65536", "mixed4096"])
def test_height_workloads_against_oracle(qfs, name):
    F, P, H = load_golden(name)
    say("height workload %s (%d surfaces)" % (name, len(H)))
    got = host(qfs.height(dev(F), dev(P), max_p=int(P.max())))
    bad = np.flatnonzero(got != H)
    assert bad.size == 0, "%d of %d heights differ; first %s: got %s want %s" % (
        bad.size, len(H), bad[:5], got[bad[:5]], H[bad[:5]])


@pytest.mark.parametrize("name", ["p5_single", "p7_single", "p5_batch8192", "p7_batch65536", "mixed4096"])
def test_height_reduced_workloads_against_oracle(qfs, name):
    # the reduced form (one 35 x 35 linear map per deep surface) against the
    # heights Algorithm 3's C tier stored for the workload
    F, P, H = load_golden(name)
    say("height_reduced workload %s (%d surfaces)" % (name, len(H)))
    got = host(qfs.height_reduced(dev(F), dev(P), max_p=int(P.max())))
    bad = np.flatnonzero(got != H)
    assert bad.size == 0, "%d of %d heights differ; first %s: got %s want %s" % (
        bad.size, len(H), bad[:5], got[bad[:5]], H[bad[:5]])


def test_mfma_peak_is_plausible(qfs):
    # the measured int8 matrix-core rate lies below the nominal dense peak (5.0 POP/s)
    say("mfma peak loop")
    tops = qfs.mfma_peak(2000)
    assert 500.0 < tops < 5000.0 * 1.05


def test_height_census_sample_against_oracle(qfs):
    # a sample of the census workload (coefficients uniform in F_5): every height from the
    # reduced path and from qfs_height equals the oracle's
    F = workloads.uniform(5, 2048, seed=1000)
    P = np.full(len(F), 5, dtype=np.int32)
    say("census sample p=5 (2048 uniform quartics)")
    want = fast.heights(F, P)
    assert host(qfs.height_reduced(dev(F), 5)).tolist() == list(want)
    assert host(qfs.height(dev(F), 5)).tolist() == list(want)


@pytest.mark.parametrize("p", [5, 7, 11])
def test_height_reduced_paper_tables(qfs, p):
    F, H = paper_rows(p)
    say("height_reduced paper table p=%d" % p)
    assert host(qfs.height_reduced(dev(F), p)).tolist() == H.tolist()


@pytest.mark.parametrize("bound", [1, 2, 3, 5])
def test_height_reduced_bounds_match_height(qfs, bound):
    # every bound gives the heights of Algorithm 3 cut at that bound
    F, P, H = load_golden("mixed4096")
    want = np.where((H >= 1) & (H <= bound), H, 0)
    say("height_reduced bound %d on mixed4096" % bound)
    got = host(qfs.height_reduced(dev(F), dev(P), bound=bound, max_p=int(P.max())))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("name", ["p5_single", "p7_single"])
def test_height_plain_against_oracle(qfs, name):
    F, P, H = load_golden(name)
    say("height_plain workload %s" % name)
    got = host(qfs.height_plain(dev(F), int(P[0])))
    assert got.tolist() == H.tolist()


def test_height_plain_paper_table_p5(qfs):
    F, H = paper_rows(5)
    say("height_plain paper table p=5")
    assert host(qfs.height_plain(dev(F), 5)).tolist() == H.tolist()


def test_height_edge_cases(qfs):
    p = 7
    F = workloads.config_p7_single(0, 4)[0]
    F = np.concatenate([F, np.zeros((1, 35), np.uint8), workloads.fermat()[None]])
    F_bad = F.copy()
    F_bad[0, 0] = 7
    P = np.full(len(F), 7, np.int32)
    P_bad = P.copy()
    P_bad[2] = 13
    want = np.array([fast.height(f, p) for f in F], dtype=np.int32)
    say("height edge cases")
    assert host(qfs.height(dev(F), p)).tolist() == want.tolist()
    assert want[4] == 0  # f = 0: g = 0, Delta = 0, never leaves m^[p]
    got = host(qfs.height(dev(F_bad), dev(P_bad), max_p=7))
    assert got[0] == qfs.QFS_EINVAL and got[2] == qfs.QFS_EUNSUPPORTED
    assert got[[1, 3, 4, 5]].tolist() == want[[1, 3, 4, 5]].tolist()
    # a prime above max_p is rejected per surface
    F5 = workloads.bernoulli_support(5, 2, 0.8, seed=55)
    got = host(qfs.height(dev(F5), dev(np.array([7, 5], np.int32)), max_p=5))
    assert got[0] == qfs.QFS_EUNSUPPORTED and got[1] == fast.height(F5[1], 5)
    # bound: b = 1 classifies every deep surface as infinite; b = 2 stops after one theta
    for b in (1, 2, 3):
        wb = np.array([fast.height(f, p, b) for f in F], dtype=np.int32)
        assert host(qfs.height(dev(F), p, bound=b)).tolist() == wb.tolist()
    # a batch of one and an empty batch
    assert host(qfs.height(dev(F[5:6]), p)).tolist() == [want[5]]
    assert qfs.height(dev(F[:0]), p).numel() == 0


def test_height_invariant_under_variable_permutation(qfs):
    F, P, H = load_golden("p5_batch8192")
    F, H = F[:512], H[:512]
    perm = (2, 0, 3, 1)
    B4 = workloads.B4
    idx = [B4.index(tuple(e[perm[j]] for j in range(4))) for e in B4]
    Fp = np.zeros_like(F)
    Fp[:, idx] = F
    say("height invariance under permutation")
    assert host(qfs.height(dev(Fp), 5)).tolist() == H.tolist()


def test_height_deterministic(qfs):
    F, P, H = load_golden("p5_batch8192")
    say("height determinism")
    a = host(qfs.height(dev(F), 5))
    b = host(qfs.height(dev(F), 5))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("name", ["p5_batch8192", "p7_single", "p7_batch65536", "mixed4096"])
def test_height_band_pass_matches_full_chain(qfs, name):
    # the capped chain decides h = 2 from the window of Delta_1 the first test
    # reads; with it switched off every deep surface runs the full chain
    F, P, H = load_golden(name)
    say("height with and without the capped chain: %s" % name)
    qfs.set_option("height_band", 0)
    try:
        full = host(qfs.height(dev(F), dev(P), max_p=int(P.max())))
    finally:
        qfs.set_option("height_band", 1)
    band = host(qfs.height(dev(F), dev(P), max_p=int(P.max())))
    assert np.array_equal(full, H)
    assert np.array_equal(band, H)


@pytest.mark.parametrize("name", ["p5_batch8192", "p7_batch65536"])
def test_height_bound_two_on_workloads(qfs, name):
    # with b = 2 Algorithm 3 returns h for h <= 2 and infinity otherwise: the
    # capped chain alone decides every deep surface
    F, P, H = load_golden(name)
    want = np.where((H == 1) | (H == 2), H, 0)
    say("height bound 2: %s" % name)
    got = host(qfs.height(dev(F), dev(P), bound=2, max_p=int(P.max())))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("name", ["p5_batch8192", "mixed4096"])
def test_height_graph_replays_match_direct_launches(qfs, name):
    # the second call with the same arguments captures the launch sequence into
    # a hipGraph; later calls replay it.  Between replays the program does its
    # own eager GPU work and synchronizes; every replay must equal the direct result.
    F, P, H = load_golden(name)
    f, pt = dev(F), dev(P)
    maxp = int(P.max())
    ws = qfs.Workspace()
    out = torch.empty(len(H), dtype=torch.int32, device="cuda")
    say("height graph replays: %s" % name)
    qfs.set_option("height_graph", 0)
    try:
        direct = host(qfs.height(f, pt, max_p=maxp, workspace=ws, out=out)).copy()
    finally:
        qfs.set_option("height_graph", 1)
    assert np.array_equal(direct, H)
    before = qfs.get_option("height_graphs_cached")
    for rep in range(5):
        out.fill_(-7)
        got = host(qfs.height(f, pt, max_p=maxp, workspace=ws, out=out)).copy()
        assert np.array_equal(got, direct), "replay %d differs" % rep
        # unrelated eager work on the same stream between replays
        x = torch.randn(512, 512, device="cuda")
        (x @ x).sum().item()
        torch.cuda.synchronize()
    assert qfs.get_option("height_graphs_cached") >= min(before + 1, 8)


def test_autotune_keeps_heights_and_stores_its_choice(qfs, tmp_path):
    F, P, H = load_golden("p5_batch8192")
    cache = str(tmp_path / "tune.jsonl")
    say("autotune p5_batch8192")
    try:
        got = host(qfs.autotune(dev(F), dev(P), max_p=5, cache_path=cache, reps=1))
        assert np.array_equal(got, H)
        chosen = (qfs.get_option("deep_slots"), qfs.get_option("gpow_per_cu"))
        lines = open(cache).read().strip().splitlines()
        assert len(lines) == 1
        rec = json.loads(lines[0])
        assert (rec["deep_slots"], rec["gpow_per_cu"]) == chosen and len(rec["trials_ms"]) == 9
        # heights under the chosen setting, and after reloading it from the file
        assert np.array_equal(host(qfs.height(dev(F), dev(P), max_p=5)), H)
        qfs.set_option("deep_slots", 0)
        qfs.set_option("gpow_per_cu", 8)
        qfs.load_tuning(cache, 5)
        assert (qfs.get_option("deep_slots"), qfs.get_option("gpow_per_cu")) == chosen
        assert np.array_equal(host(qfs.height(dev(F), dev(P), max_p=5)), H)
    finally:
        qfs.set_option("deep_slots", 0)
        qfs.set_option("gpow_per_cu", 8)
