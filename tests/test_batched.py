"""GPU parity of the batched persistent FP64 protected GEMM (many uneven problems in
one launch per tile configuration), through the C ABI, against the CPU oracle.

Each problem must match the oracle's plain triple loop within the componentwise
rounding bound; with per-problem injection, the injection log of every problem
must reproduce the plan the oracle derives from that problem's seed, and the
located elements must agree with the oracle's simulation of the same plan.
A hipGraph capture of the call must replay to the eager result."""
import numpy as np
import pytest

import oracle
from paper_2104_00897_amd import inputs
from tests.gpu_util import assert_close_f64, magnitude

pytestmark = pytest.mark.gpu

TILE_SHAPE = {2: (128, 128), 3: (64, 64)}


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2104_00897_amd import ftgemm
    assert torch.cuda.is_available()
    h = ftgemm.Handle(capacity=16384)
    yield ftgemm, h, torch
    torch.cuda.synchronize()
    h.close()


def problem_seed(seed, p):
    """Seed of problem p's injector (documented with the batched entry point)."""
    return oracle.splitmix64(seed, 2 ** 32 + p)


class Batch:
    """Host operands (Fortran order), device copies, and the argument plan."""

    def __init__(self, env, specs, seed):
        ftgemm, _, torch = env
        self.specs = specs
        self.host, self.dev, probs = [], [], []
        for q, (m, n, k, ta, tb, alpha, beta) in enumerate(specs):
            A, B, C = inputs.gemm_operands_f64(m, n, k, seed=seed * 1000 + q, ta=ta, tb=tb)
            dA, dB = ftgemm.to_device(A), ftgemm.to_device(B)
            if beta == 0.0:
                dC = torch.full((n, m), float("nan"), dtype=torch.float64, device="cuda")
            else:
                dC = ftgemm.to_device(C)
            self.host.append((A, B, C))
            self.dev.append((dA, dB, dC))
            probs.append(ftgemm.batch_problem(dA, dB, dC, alpha, beta, ta, tb))
        self.pristine = [d[2].clone() for d in self.dev]
        self.plan = ftgemm.BatchPlan(probs)

    def restore(self):
        for d, c in zip(self.dev, self.pristine):
            d[2].copy_(c)

    def outputs(self, ftgemm):
        return [ftgemm.to_host(d[2]) for d in self.dev]

    def reference(self, q):
        m, n, k, ta, tb, alpha, beta = self.specs[q]
        A, B, C = self.host[q]
        return oracle.gemm(A, B, C if beta else None, alpha, beta, ta, tb)


def run(env, batch, cfg=None, faults=None):
    ftgemm, h, torch = env
    batch.restore()
    h.reset()
    h.dgemm_batched(batch.plan, ftgemm.current_stream_ptr(), cfg, faults)
    torch.cuda.synchronize()
    return batch.outputs(ftgemm), h.read()


def mixed_specs(rng, count):
    specs = []
    ab = [(1.0, 0.0), (1.5, 0.5), (-2.0, 1.0), (0.75, -1.25)]
    for _ in range(count):
        m, n, k = (int(x) for x in rng.integers(1, 330, size=3))
        ta, tb = (int(x) for x in rng.integers(0, 2, size=2))
        alpha, beta = ab[int(rng.integers(0, len(ab)))]
        specs.append((m, n, k, ta, tb, alpha, beta))
    # edge cases: single element, exact tiles, k = 0, alpha = 0, empty problems
    specs += [(1, 1, 1, 0, 0, 1.0, 0.0), (64, 64, 64, 0, 0, 1.0, 0.5), (128, 256, 129, 1, 1, 1.5, 0.5),
              (65, 1, 300, 0, 1, 1.0, 0.0), (40, 30, 0, 0, 0, 1.0, 0.5), (50, 20, 70, 0, 0, 0.0, 2.0),
              (0, 20, 10, 0, 0, 1.0, 0.0), (20, 0, 10, 0, 0, 1.0, 0.0), (33, 17, 25, 1, 0, 0.0, 1.0)]
    return specs


@pytest.mark.parametrize("tile", [0, 2, 3])
def test_batched_fault_free_mixed(env, tile):
    ftgemm = env[0]
    specs = mixed_specs(np.random.default_rng(31 + tile), 40)
    batch = Batch(env, specs, seed=5)
    outs, rep = run(env, batch, ftgemm.make_config(tile=tile))
    for q, (m, n, k, ta, tb, alpha, beta) in enumerate(specs):
        if m == 0 or n == 0:
            continue
        A, B, C = batch.host[q]
        ref = batch.reference(q)
        if k == 0 or alpha == 0.0:
            np.testing.assert_array_equal(outs[q], ref if beta else np.zeros((m, n)))
            continue
        assert_close_f64(outs[q], ref, magnitude(A, B, C, alpha, beta, ta, tb), k)
    assert rep.detected == 0 and rep.records == []


def test_batched_unprotected_and_integer_bitwise(env):
    ftgemm, h, torch = env
    rng = np.random.default_rng(12)
    specs, host, probs, dev = [], [], [], []
    for q in range(16):
        m, n, k = (int(x) for x in rng.integers(20, 260, size=3))
        A, B, C = inputs.integer_operands(m, n, k, seed=100 + q)
        dA, dB, dC = ftgemm.to_device(A), ftgemm.to_device(B), ftgemm.to_device(C)
        specs.append((m, n, k)); host.append((A, B, C)); dev.append((dA, dB, dC))
        probs.append(ftgemm.batch_problem(dA, dB, dC, 1.5, -2.0))
    pristine = [d[2].clone() for d in dev]
    plan = ftgemm.BatchPlan(probs)
    for abft in (True, False):
        for d, c in zip(dev, pristine):
            d[2].copy_(c)
        h.dgemm_batched(plan, ftgemm.current_stream_ptr(), ftgemm.make_config(abft=abft))
        torch.cuda.synchronize()
        for (A, B, C), d in zip(host, dev):
            np.testing.assert_array_equal(ftgemm.to_host(d[2]), oracle.gemm(A, B, C, 1.5, -2.0))


def check_faults(batch, rep, faults, seed, tile, bit_lo, bit_hi, kc=0):
    """Per problem: injection log == oracle plan; located elements == oracle.abft's."""
    bm, bn = TILE_SHAPE[tile]
    total = 0
    for q, (m, n, k, ta, tb, alpha, beta) in enumerate(batch.specs):
        plan = oracle.fault_plan(problem_seed(seed, q), int(faults[q]), m, n, k, bm, bn, kc=kc,
                                 kgran=128, bit_lo=bit_lo, bit_hi=bit_hi)
        total += len(plan)
        got = sorted((r["row"], r["col"], r["pflip"], r["bit"]) for r in rep.inject_log if r["problem"] == q)
        want = sorted((f.tile_m * bm + f.row, f.tile_n * bn + f.col, f.pflip, f.bit) for f in plan)
        assert got == want, (q, got, want)
        located = sorted((r["interval"], r["row"], r["col"]) for r in rep.records if r["problem"] == q)
        A, B, C = batch.host[q]
        _, orecs, _ = oracle.abft(A, B, C if beta else None, alpha, beta, ta, tb, bm=bm, bn=bn, kc=kc,
                                  plan=plan)
        assert located == sorted((r.interval, r.row, r.col) for r in orecs), q
    return total


@pytest.mark.parametrize("tile", [2, 3])
def test_batched_faults_per_problem(env, tile):
    """0-2 faults per problem (U{0,1,2}), exponent and high mantissa bits: every
    fault is located where the plan put it and corrected."""
    ftgemm = env[0]
    rng = np.random.default_rng(7)
    specs = []
    for _ in range(24):
        m, n = (int(x) for x in rng.integers(70, 400, size=2))   # >= 2 tiles of 64 x 64
        k = int(rng.integers(1, 400))
        specs.append((m, n, k, 0, 0, 1.5, 0.5))
    faults = rng.integers(0, 3, size=len(specs))
    batch = Batch(env, specs, seed=6)
    cfg = ftgemm.make_config(tile=tile, seed=7, n_faults=1, bit_lo=52, bit_hi=62)
    outs, rep = run(env, batch, cfg, faults)
    total = check_faults(batch, rep, faults, 7, tile, 52, 62)
    assert rep.injected == total
    assert rep.corrected_subtract + rep.corrected_recompute == total and rep.uncorrectable == 0
    for q, (m, n, k, ta, tb, alpha, beta) in enumerate(specs):
        A, B, C = batch.host[q]
        assert_close_f64(outs[q], batch.reference(q), magnitude(A, B, C, alpha, beta, ta, tb), k)


def test_batched_interval_mode(env):
    """Small problems (one tile) take two faults through 128-step verification intervals."""
    ftgemm = env[0]
    rng = np.random.default_rng(8)
    specs = [(int(rng.integers(20, 64)), int(rng.integers(20, 64)), int(rng.integers(300, 700)), 0, 0, 1.0, 0.0)
             for _ in range(20)]
    faults = np.full(len(specs), 2)
    batch = Batch(env, specs, seed=7)
    cfg = ftgemm.make_config(tile=3, interval_k=128, seed=9, n_faults=2, bit_lo=52, bit_hi=62)
    outs, rep = run(env, batch, cfg, faults)
    total = check_faults(batch, rep, faults, 9, 3, 52, 62, kc=128)
    assert total == 2 * len(specs) and rep.injected == total
    assert rep.corrected_subtract + rep.corrected_recompute == total
    for q, (m, n, k, ta, tb, alpha, beta) in enumerate(specs):
        A, B, C = batch.host[q]
        assert_close_f64(outs[q], batch.reference(q), magnitude(A, B, C, alpha, beta, ta, tb), k)


def test_batched_graph_replay(env):
    """A captured batched call (report reset + copy + persistent kernel + repair)
    replays to the eager result, with eager work and synchronisation between replays."""
    ftgemm, h, torch = env
    rng = np.random.default_rng(11)
    specs = [(int(rng.integers(40, 300)), int(rng.integers(40, 300)), int(rng.integers(1, 300)), 0, 0, 1.5, 0.5)
             for _ in range(30)]
    faults = rng.integers(0, 3, size=len(specs))
    batch = Batch(env, specs, seed=8)
    cfg = ftgemm.make_config(tile=3, seed=5, n_faults=1, bit_lo=52, bit_hi=62)
    eager, rep0 = run(env, batch, cfg, faults)
    assert rep0.injected == rep0.corrected_subtract + rep0.corrected_recompute
    batch.restore()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        h.reset(ftgemm.current_stream_ptr())
        h.dgemm_batched(batch.plan, ftgemm.current_stream_ptr(), cfg, faults)
    torch.cuda.synchronize()
    for _ in range(3):
        batch.restore()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        outs = batch.outputs(ftgemm)
        for q in range(len(specs)):
            np.testing.assert_array_equal(outs[q], eager[q])
        rep = h.read()
        assert (rep.injected, rep.corrected_subtract, rep.corrected_recompute) == \
               (rep0.injected, rep0.corrected_subtract, rep0.corrected_recompute)
        # eager work on the same handle between replays
        h.dgemm_batched(batch.plan, ftgemm.current_stream_ptr(), ftgemm.make_config(abft=False))
        torch.cuda.synchronize()
    del g


def test_batched_argument_errors(env):
    ftgemm, h, torch = env
    d = torch.zeros(64, dtype=torch.float64, device="cuda")
    good = dict(ta=0, tb=0, m=4, n=4, k=4, alpha=1.0, beta=0.0, A=d.data_ptr(), lda=4,
                B=d.data_ptr(), ldb=4, C=d.data_ptr(), ldc=4)
    for bad, info in [(dict(lda=3), 8), (dict(ldb=3), 10), (dict(ldc=2), 13), (dict(m=-1), 3),
                      (dict(ta=5), 1)]:
        plan = ftgemm.BatchPlan([good, {**good, **bad}])
        with pytest.raises(ftgemm.FtgError) as e:
            h.dgemm_batched(plan)
        assert e.value.status == ftgemm.ERR_INVALID_ARG and e.value.info == info
    with pytest.raises(ftgemm.FtgError) as e:
        h.dgemm_batched(ftgemm.BatchPlan([good]), cfg=ftgemm.make_config(tile=1))
    assert e.value.status == ftgemm.ERR_UNSUPPORTED
    big = ftgemm.BatchPlan([good] * 1500)
    with pytest.raises(ftgemm.FtgError) as e:
        h.dgemm_batched(big)
    assert e.value.status == ftgemm.ERR_UNSUPPORTED
    h.batched_reserve(2048)
    h.dgemm_batched(big)
    torch.cuda.synchronize()


def cfg5_specs(count=512, seed=7, lo=32, hi=2048):
    sizes = inputs.log_uniform_sizes(count, lo, hi, seed)
    return [(int(m), int(n), int(k), 0, 0, 1.0, 0.0) for m, n, k in sizes]


def test_batched_cfg5_full_size_sampled(env):
    """512 problems with m, n, k log-uniform in [32, 2048] (seed 7), 0-2 faults per
    problem at the default bits 40..63: sampled entries of every problem and every
    faulted element against the oracle; faults of detectable size are corrected."""
    ftgemm, h, torch = env
    specs = cfg5_specs()
    rng = np.random.default_rng(7)
    faults = rng.integers(0, 3, size=len(specs))
    batch = Batch(env, specs, seed=9)
    cfg = ftgemm.make_config(tile=3, seed=7, n_faults=1)
    outs, rep = run(env, batch, cfg, faults)
    assert rep.uncorrectable == 0
    assert rep.detected == rep.corrected_subtract + rep.corrected_recompute + rep.checksum_only
    fixed = {(r["problem"], r["row"], r["col"]) for r in rep.records if r["kind"] in (1, 2)}
    n_inj = 0
    for q, (m, n, k, ta, tb, alpha, beta) in enumerate(specs):
        A, B, _ = batch.host[q]
        inj = [r for r in rep.inject_log if r["problem"] == q]
        n_inj += len(inj)
        rows = list(rng.integers(0, m, size=12)) + [r["row"] for r in inj]
        cols = list(rng.integers(0, n, size=12)) + [r["col"] for r in inj]
        ref = oracle.gemm_entries(A, B, None, rows, cols, alpha, beta, ta, tb)
        got = outs[q][rows, cols]
        mag = np.abs(A)[rows, :] * np.abs(B)[:, cols].T
        M = mag.sum(axis=1) * abs(alpha)
        tol = max(1e-12, 2.2 * k * 2.0 ** -53) * M
        for e, r in enumerate(inj):
            x = len(rows) - len(inj) + e
            if (q, r["row"], r["col"]) in fixed:
                continue
            # undetected: the flip was below the threshold (masked); its effect stays bounded
            d = abs(r["new_val"] - r["old_val"]) * abs(alpha)
            assert abs(got[x] - ref[x]) <= d * 1.01 + tol[x], (q, r)
            tol[x] = np.inf
        bad = np.abs(got - ref) > tol
        assert not bad.any(), (q, np.argwhere(bad)[:3])
    # F_p is capped by the problem's slot count (one-tile problems take at most one)
    expect = sum(min(int(f), -(-m // 64) * -(-n // 64)) for f, (m, n, *_) in zip(faults, specs))
    assert rep.injected == n_inj == expect


def test_batched_encode_pass_and_in_loop_agree(env):
    """Batched calls with the encode pass (default) and with the encode inside the
    k loop locate the same faults and both match the oracle."""
    ftgemm = env[0]
    rng = np.random.default_rng(21)
    specs = [(int(rng.integers(70, 300)), int(rng.integers(70, 300)), int(rng.integers(1, 400)),
              int(rng.integers(0, 2)), int(rng.integers(0, 2)), 1.5, 0.5) for _ in range(20)]
    faults = rng.integers(0, 3, size=len(specs))
    batch = Batch(env, specs, seed=10)
    got = []
    for in_loop in (False, True):
        cfg = ftgemm.make_config(tile=3, seed=3, n_faults=1, bit_lo=52, bit_hi=62, encode_in_loop=in_loop)
        outs, rep = run(env, batch, cfg, faults)
        assert rep.injected == rep.corrected_subtract + rep.corrected_recompute
        for q, (m, n, k, ta, tb, alpha, beta) in enumerate(specs):
            A, B, C = batch.host[q]
            assert_close_f64(outs[q], batch.reference(q), magnitude(A, B, C, alpha, beta, ta, tb), k)
        got.append(sorted((r["problem"], r["row"], r["col"], r["kind"]) for r in rep.records))
    assert got[0] == got[1]
