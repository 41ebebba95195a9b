"""Host logic of the autotuner (no GPU): coordinate descent keeps the fastest
setting, every setting it tries must return the reference result, and the
time budget ends the search.  The workload is a stand-in whose speed depends
on the parameters; device synchronization is stubbed out."""
import time

import pytest
import torch

from paper_2108_01731_amd import autotune as T
from paper_2108_01731_amd import lcc as L

SPACE = {"queue_ahead": [0, 1, 4], "score_pruning": [0, 1, -1]}


@pytest.fixture(autouse=True)
def no_device_sync(monkeypatch):
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)


def fake_workload(slow_ms, key_of=lambda p: "same"):
    """run(params): sleeps slow_ms(params) milliseconds, returns key_of(params)."""
    calls = []

    def run(prm):
        calls.append((prm.queue_ahead, prm.score_pruning))
        time.sleep(slow_ms(prm) / 1e3)
        return key_of(prm)

    return run, calls


def test_descent_keeps_the_fastest_setting_of_each_field():
    # queue_ahead = 4 and score_pruning = -1 are fast, the rest slow
    def slow(p):
        return 2.0 + (0.0 if p.queue_ahead == 4 else 25.0) + (0.0 if p.score_pruning == -1 else 25.0)

    run, calls = fake_workload(slow)
    best, table = T.tune(run, space=SPACE, reps=1, budget_s=60.0)
    assert (best.queue_ahead, best.score_pruning) == (4, -1)
    # the reference plus every other value of each field, one field at a time
    assert len(table) == 1 + 2 + 2
    assert calls[0] == (0, 0)
    # the second field is searched from the first field's winner
    assert all(qa == 4 for qa, _ in calls[3:])
    assert table[0]["params"] == {"queue_ahead": 0, "score_pruning": 0}


def test_a_setting_that_changes_the_result_raises():
    run, _ = fake_workload(lambda p: 1.0, key_of=lambda p: "other" if p.score_pruning == 1 else "same")
    with pytest.raises(T.TuningChangedResult, match="score_pruning=1"):
        T.tune(run, space=SPACE, reps=1, budget_s=60.0)


def test_repeated_runs_must_agree():
    state = {"n": 0}

    def key_of(p):
        state["n"] += 1
        return str(state["n"])  # a different result on every run

    run, _ = fake_workload(lambda p: 0.5, key_of=key_of)
    with pytest.raises(T.TuningChangedResult, match="repeated runs"):
        T.tune(run, space=SPACE, reps=2, budget_s=60.0)


def test_the_budget_ends_the_search_with_the_best_so_far():
    run, calls = fake_workload(lambda p: 1.0)
    best, table = T.tune(run, base=L.Params(), space=SPACE, reps=1, budget_s=0.0)
    assert len(calls) == 1 and len(table) == 1
    assert (best.queue_ahead, best.score_pruning) == (0, 0)


def test_result_key_depends_on_labels_and_numerators():
    a = torch.arange(10, dtype=torch.int32)
    b = a.clone()
    b[3] = 7
    assert T.result_key(a, 5) == T.result_key(a.clone(), 5)
    assert T.result_key(a, 5) != T.result_key(b, 5)
    assert T.result_key(a, 5) != T.result_key(a, 6)
