"""Race check of the generalized eigenproblem reduction's stream schedule
(host only: runs here without a GPU).

hs_gep_check_schedule runs the library's own orchestration of the
reduction without issuing anything, records every launch with its stream
and the cells of each matrix it reads and writes, and every event record
and stream wait, and counts the pairs of launches on different streams that
touch a common 128 x 128 cell, one of them writing, with no chain of stream
order and event waits between them.

The schedule must be free of such pairs at every size (the lookahead from
4 panels, the background stream from 8, the two-term Ht from N = 4096) and
in both arithmetic modes. Leaving out one wait site at a time must open a
race, which shows that the check sees each dependency. The one exception
is site 6, the factorization's final join of the transposes stream: in a
run without errors every transpose is already consumed (and waited for) by
the panel that follows it, so that join only orders work on an error path.
"""

import pytest

import paper_1611_00606_amd as P

SIZES = [1, 2, 127, 128, 129, 385, 513, 897, 1025, 1500, 4095, 4096, 4200, 8000, 16000]


@pytest.mark.parametrize("mode", [P.HS_FP64, P.HS_FP64_3M])
@pytest.mark.parametrize("N", SIZES)
def test_schedule_is_race_free(N, mode):
    n, report = P.hs_gep_check_schedule(N, mode)
    assert n == 0, report


# wait sites (see hs_gep_check_schedule): 1 next S21^H after the next column
# block, 2 panel product after S21^H, 3 next column block after the previous
# bulk update, 4 lookahead after the panel product, 5 final join of the
# lookahead stream, 7 background fork after the top split's panel, 8
# background after the pending lookahead work, 9 top split's M21 after the
# leading block's inverse, 10 Ht's last rows after the background products
@pytest.mark.parametrize("N", [1500, 4200])
@pytest.mark.parametrize("site", [1, 2, 3, 4, 5, 7, 8, 9, 10])
def test_each_missing_wait_is_found(N, site):
    n, report = P.hs_gep_check_schedule(N, P.HS_FP64, drop_wait=site)
    assert n > 0
    assert " and " in report and "cell" in report


def test_final_transpose_join_orders_only_error_paths():
    for N in (1500, 4200):
        assert P.hs_gep_check_schedule(N, P.HS_FP64, drop_wait=6)[0] == 0


def test_background_fork_needs_the_lookahead_wait():
    """Without the background stream's wait for the lookahead stream, the
    last L21 transpose before the top split still reads LH columns that the
    background's V (or WH) product overwrites."""
    for N in (1500, 4200):
        n, report = P.hs_gep_check_schedule(N, P.HS_FP64, drop_wait=8)
        assert n > 0 and "k_gep_conj_t" in report and "LH" in report


def test_arguments():
    assert P.hs_gep_check_schedule(0)[0] == -1
    assert P.hs_gep_check_schedule(100, P.HS_SPLIT_F16)[0] == -2
    assert P.hs_gep_check_schedule(100, 7)[0] == -2
