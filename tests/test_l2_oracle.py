"""Pins of the L2 / NRMSE-bounded oracle (oracle.l2), on the CPU (their
bodies live in oracle_pins.py, so that the planted slips of
test_oracle_mutations.py are checked against them too):

* Eckart-Young: the eigenvalue tail after r modes equals the squared
  Frobenius error of the rank-r projection, computed directly;
* the hand-worked one-block fields of tests/golden/l2_block_2x2.json
  (budget, rank, step, quantized basis and coefficients, decoded values,
  error) and the rank rule's hand cases;
* the block budgets add up to the variable's squared global budget;
* every block's exact error within its budget and every variable's NRMSE
  within its target on blob and drifting-spectrum fields (1e-1 .. 1e-4),
  stream round trip bit for bit, the precision parameter without effect;
* ranks grow as the target tightens; non-finite, zero and too-tight blocks.
"""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle_pins as P  # noqa: E402


def test_eckart_young_tail_is_projection_error():
    P.pin_l2_eckart_young()


def test_hand_worked_blocks():
    P.pin_l2_hand_case()


def test_budgets_add_up_to_the_global_budget():
    P.pin_l2_budgets_sum()


@pytest.mark.parametrize("target", [1e-1, 1e-2, 1e-3, 1e-4])
def test_every_block_within_budget_and_nrmse_within_target(target):
    P.pin_l2_bound_and_round_trip((target,))


def test_ranks_grow_as_the_target_tightens():
    P.pin_l2_ranks_grow()


def test_special_blocks():
    P.pin_l2_special_blocks()
