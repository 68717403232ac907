"""Per-iteration records of a solver history (history_records, the JSONL
log): the inertial weights follow the t recurrence of Alg. 4, losses that
were not formed stay empty, and decreases and steps are read off the
history."""
import json
import math

import numpy as np

from paper_2506_04045_amd import history_records


def _hist(k, f=None):
    rng = np.random.default_rng(0)
    f = np.cumsum(-rng.random(k + 1)) + 100.0 if f is None else np.asarray(f, float)
    return dict(f=f, tau=np.full(k + 1, 0.25), trials=np.ones(k + 1, np.int32),
                r=np.linspace(1.0, 0.1, k + 1))


def test_fista_weights_follow_the_t_recurrence():
    recs = history_records(_hist(40), accelerate=True)
    beta = [r["beta"] for r in recs[1:]]
    assert beta[0] == 0.0 and beta[1] == 0.0          # Y_1 = Xbar_0, t_1 = 1
    t2 = (1 + math.sqrt(5)) / 2
    t3 = (1 + math.sqrt(1 + 4 * t2 * t2)) / 2
    assert beta[2] == (t2 - 1) / t3
    assert all(b1 > b0 for b0, b1 in zip(beta[2:], beta[3:])) and beta[-1] < 1.0
    # t_n >= (n + 1) / 2 gives beta_n >= (n - 3) / (n + 1)... and beta_n -> 1
    for n, b in enumerate(beta, start=1):
        if n >= 3:
            assert b >= (n - 3) / (n + 1) - 1e-15


def test_gpa_has_no_inertia_and_fields_are_read_off_the_history():
    h = _hist(5)
    recs = history_records(h, accelerate=False)
    assert [r["iter"] for r in recs] == list(range(6))
    assert recs[0] == {"iter": 0, "f": h["f"][0]}
    for n in range(1, 6):
        r = recs[n]
        assert r["beta"] == 0.0 and r["tau"] == 0.25 and r["L"] == 4.0 and r["trials"] == 1
        assert r["df"] == h["f"][n - 1] - h["f"][n] and r["pgrad"] == h["r"][n]


def test_losses_not_formed_stay_empty():
    f = [10.0, math.nan, math.nan, 7.0, 6.5]
    recs = history_records(_hist(4, f), accelerate=True)
    assert [r["f"] for r in recs] == [10.0, None, None, 7.0, 6.5]
    assert [r.get("df") for r in recs[1:]] == [None, None, None, 0.5]
    json.dumps(recs, allow_nan=False)   # valid JSON, no NaN tokens
