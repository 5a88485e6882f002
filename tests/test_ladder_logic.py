"""Host logic of the precision ladder (gn_ladder_to_target), without a GPU: the Gauss-Newton
optimizer is replaced by a stand-in whose residual sequence per storage form is scripted, so the
acceptance, rejection, restore and switching rules can be checked exactly."""
import pytest

torch = pytest.importorskip("torch")

from paper_1910_12331_amd import api, optim  # noqa: E402


class FakeTensor:
    """Storage form stand-in: a name and the residuals its steps produce, in order."""

    def __init__(self, name, residuals, start):
        self.name, self.residuals, self.start = name, list(residuals), start


@pytest.fixture
def fake(monkeypatch):
    log = []

    class FakeGN:
        def __init__(self, X, A, config):
            self.X, self.A, self.cfg, self.k = X, list(A), config, 0
            self.schedule = config.schedule
            self.r = X.start

        def step(self):
            self.r = self.X.residuals[self.k]
            self.k += 1
            for a in self.A:
                a.add_(1.0)             # every step moves the factors
            self.schedule.advance()
            log.append((self.X.name, self.r))

        def residual(self):
            return self.r

    monkeypatch.setattr(optim, "GaussNewton", FakeGN)
    monkeypatch.setattr(optim, "_rung_name", lambda X: X.name)
    monkeypatch.setattr(optim.api, "factor_dtype", lambda X: torch.float32)
    return log


def test_rejected_step_restores_and_moves_up(fake):
    low = FakeTensor("bf16", [0.3, 0.1, 0.05, 1e9], start=1.0)
    top = FakeTensor("torch.float64", [1e-2, 1e-3], start=0.05)
    A = [torch.zeros(3, 2)]
    sched = optim.DampingSchedule()
    out, hist = optim.gn_ladder_to_target([low, top], A, 2e-3, optim.GNConfig(schedule=sched))
    assert [h[:1] + h[2:] for h in hist] == [("bf16", True)] * 3 + [("bf16", False)] + \
        [("torch.float64", True)] * 2
    # three accepted low steps and two top steps moved the factors; the rejected one did not
    assert torch.equal(out[0], torch.full((3, 2), 5.0))
    # the damping schedule advanced once per accepted step only
    ref = optim.DampingSchedule()
    for _ in range(5):
        ref.advance()
    assert sched.value == ref.value and sched.decreasing == ref.decreasing


def test_floor_and_stall_switch_up(fake):
    low = FakeTensor("bf16", [0.5, 0.009, 0.0085], start=1.0)           # 0.009 <= floor 1e-2
    mid = FakeTensor("bf16x3", [4e-3, 2.5e-3], start=0.009)   # 2.5e-3: no halving, < 100 floor
    top = FakeTensor("torch.float64", [1e-3, 5e-4], start=2.5e-3)
    A = [torch.zeros(2, 2)]
    _, hist = optim.gn_ladder_to_target([low, mid, top], A, 6e-4)
    names = [h[0] for h in hist]
    assert names == ["bf16", "bf16", "bf16x3", "bf16x3", "torch.float64", "torch.float64"]
    assert all(ok for _, _, ok in hist) and hist[-1][1] <= 6e-4


def test_low_rung_cannot_certify_a_tighter_target(fake):
    low = FakeTensor("bf16", [1e-3], start=1.0)        # below target, but floor 1e-2 > target/10
    top = FakeTensor("torch.float64", [5e-4], start=1e-3)
    _, hist = optim.gn_ladder_to_target([low, top], [torch.zeros(1, 1)], 2e-3)
    assert [h[0] for h in hist] == ["bf16", "torch.float64"]


def test_nan_step_is_rejected(fake):
    low = FakeTensor("bf16x3", [float("nan")], start=1.0)
    top = FakeTensor("torch.float64", [1e-6], start=1.0)
    out, hist = optim.gn_ladder_to_target([low, top], [torch.zeros(1, 1)], 1e-5)
    assert hist[0][2] is False and hist[1] == ("torch.float64", 1e-6, True)
    assert torch.equal(out[0], torch.ones(1, 1))


def test_step_decay_schedule():
    """lambda = start * factor^floor(k / every) for sweep k (Section 5: 0.01, halved every 100)."""
    s = optim.StepDecay(1e-2, 0.5, 100)
    seq = [s.value]
    for _ in range(349):
        seq.append(s.advance())
    for k, v in enumerate(seq):
        assert v == 1e-2 * 0.5 ** (k // 100)
    with pytest.raises(ValueError):
        optim.StepDecay(1e-2, 0.5, 0)


def test_autotune_batched_picks_fastest_and_caches():
    """Host logic of the batched autotuner with a scripted timer (no GPU)."""
    probs = [(torch.zeros(60, 70, 90), [torch.zeros(60, 8), torch.zeros(70, 8), torch.zeros(90, 8)]),
             (torch.zeros(130, 70, 90), [torch.zeros(130, 40), torch.zeros(70, 40),
                                         torch.zeros(90, 40)])]
    secs = {(1, False, False, False): 4.0, (1, True, False, False): 3.0,
            (4, False, False, False): 2.0, (4, True, False, False): 1.0,
            (8, False, False, False): 1.5, (8, True, False, False): 1.0,
            (1, False, True, False): 2.5, (1, True, True, False): 2.5,
            (4, False, True, False): 0.8, (4, True, True, False): 0.5,
            (8, False, True, False): 0.9, (8, True, True, False): 0.5,
            (1, False, True, True): 0.6, (1, True, True, True): 0.5}
    T = api.Tiles
    # tile sweep on the chosen configuration: 8 items per wavefront wins its field (0.45 s), one
    # workgroup per CU is faster by less than the margin (0.44 s), 32-row tiles win theirs
    tile_secs = {T(4): 0.49, T(8): 0.45, T(32): 0.6, T(64): 0.7, T(8, 1): 0.44, T(8, 4): 0.5,
                 T(8, 0, 2): 0.40, T(8, 0, 4): 0.45}
    calls = []

    def timer(problems, config, ns, graphs, steps, batch_cg, fused, tiles=None):
        calls.append((ns, graphs, batch_cg, fused, tiles))
        assert problems is probs and steps == 3
        if tiles is not None:
            assert (ns, graphs, batch_cg, fused) == best_launch
            return tile_secs.get(tiles, 1.0) if best_launch == (1, True, True, True) else 1.0
        return secs[(ns, graphs, batch_cg, fused)]

    cache = {}
    best_launch = (1, True, True, True)
    out = optim.autotune_batched(probs, stream_counts=(1, 4, 8), timer=timer, cache=cache)
    # the first of the fastest (0.5 s) in sweep order: the graphed batch program
    assert (out.n_streams, out.graphs, out.batch_cg, out.fused) == best_launch
    assert len(out.table) == 14 and out.table[best_launch] == 2 * 3 / 0.5
    assert out.tiles == T(8, 0, 2) and out.problem_steps_per_s == 2 * 3 / 0.40
    assert len(out.tile_table) == 9 and out.tile_table[T()] == 2 * 3 / 0.5
    assert len(calls) == 14 + 8
    assert [c[4] for c in calls[14:]] == [T(4), T(8), T(32), T(64), T(8, 1), T(8, 4), T(8, 0, 2),
                                          T(8, 0, 4)]
    again = optim.autotune_batched(probs, stream_counts=(1, 4, 8), timer=timer, cache=cache)
    assert again is out and len(calls) == 22                  # served from the cache
    # without the batch program the batched CG on 4 streams with graphs wins; no tile shape
    # beats the default there (every tile timing is 1 s)
    best_launch = (4, True, True, False)
    out1 = optim.autotune_batched(probs, stream_counts=(1, 4, 8), timer=timer, cache={},
                                  fused=(False,))
    assert (out1.n_streams, out1.graphs, out1.batch_cg, out1.fused) == best_launch
    assert out1.tiles is None and out1.problem_steps_per_s == 2 * 3 / 0.5
    # neither batched CG nor the batch program is swept where they do not apply (the Cholesky
    # preconditioner); no tile sweep when it is switched off
    calls.clear()
    cfg = optim.GNConfig(preconditioner="cholesky")
    out2 = optim.autotune_batched(probs, cfg, stream_counts=(1, 4, 8), timer=timer, cache={},
                                  tile_sweep=False)
    assert not out2.batch_cg and not out2.fused and len(calls) == 6
    assert all(not c[2] and not c[3] and c[4] is None for c in calls)
    assert out2.tiles is None and out2.tile_table == {}
    # the bucket: ranks 8 and 40 -> 8 and 64, largest modes 90 and 130 -> 128 and 256
    assert optim.batch_key(probs) == (2, ("torch.float32",), (8, 64), (128, 256))
