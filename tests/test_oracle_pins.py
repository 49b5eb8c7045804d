import os, sys
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
"""The CPU oracle against closed forms, invariants and the paper's proxy-neuron
formulation of delay (see oracle_pins.py for the statements)."""
import pytest

from oracle_pins import ALL_PINS


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_pin(oracle, pin):
    pin(oracle)
