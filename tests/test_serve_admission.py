"""Admission rule of the serving loop (host logic, no GPU): requests that can
never run are rejected at once instead of blocking the queue, requests that
do not fit yet wait, the rest are admitted."""
from paper_2303_15491_amd.serve import ADMIT, REJECT_BATCH, REJECT_BUDGET, WAIT, admission


def test_request_above_the_whole_budget_is_rejected_not_queued():
    # fits one batch by vertex count, but its footprint exceeds the budget:
    # waiting would never help, so it must not block the queue head
    assert admission(numel=1000, nbytes=5000, resident=0, queued=0, max_vertices=10**6, budget=4096,
                     max_queued=8) == REJECT_BUDGET


def test_request_above_one_batch_is_rejected():
    assert admission(numel=2000, nbytes=100, resident=0, queued=0, max_vertices=1000, budget=10**9,
                     max_queued=8) == REJECT_BATCH


def test_request_that_fits_later_waits():
    assert admission(numel=10, nbytes=600, resident=3600, queued=0, max_vertices=1000, budget=4096,
                     max_queued=8) == WAIT
    assert admission(numel=10, nbytes=6, resident=0, queued=8, max_vertices=1000, budget=4096,
                     max_queued=8) == WAIT


def test_request_that_fits_is_admitted():
    assert admission(numel=10, nbytes=496, resident=3600, queued=7, max_vertices=1000, budget=4096,
                     max_queued=8) == ADMIT
    assert admission(numel=1000, nbytes=4096, resident=0, queued=0, max_vertices=1000, budget=4096,
                     max_queued=8) == ADMIT
