"""Planted mistakes in the fp64 network reference are caught by its pins.

Each mutant is oracle/mlp_ref.py with one plausible mistake (a dropped bias,
a missing factor, a transposed product, the wrong ReLU mask, a parameter
layout out of order, the mask left out of the loss's normalisation),
loaded as a module of its own; with it in place of the reference, at least
one pin of test_mlp_ref must fail.  CPU only.
"""
import os
import types

import numpy as np
import pytest

import test_mlp_ref as pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "mlp_ref.py")

MUTANTS = [
    ("output bias dropped", 'y = h2 @ P["W3"].T + P["b3"]', 'y = h2 @ P["W3"].T'),
    ("second bias dropped", 'z2 = h1 @ P["W2"].T + P["b2"]', 'z2 = h1 @ P["W2"].T'),
    ("second layer fed the pre-activation", 'z2 = h1 @ P["W2"].T', 'z2 = z1 @ P["W2"].T'),
    ("output passed through a ReLU", 'y = h2 @ P["W3"].T + P["b3"]', 'y = np.maximum(h2 @ P["W3"].T + P["b3"], 0.0)'),
    ("loss gradient without its factor 2", "dy = 2.0 * m * (y - t)", "dy = 1.0 * m * (y - t)"),
    ("loss normalised by all entries", "/ np.sum(m))", "/ m.size)"),
    ("W2 gradient transposed", 'g["W2"] = dz2.T @ h1', 'g["W2"] = h1.T @ dz2'),
    ("backward through W2 transposed", 'dz1 = (dz2 @ P["W2"])', 'dz1 = (dz2 @ P["W2"].T)'),
    ("ReLU mask of the wrong layer", 'dz2 = (dy @ P["W3"]) * (z2 > 0)', 'dz2 = (dy @ P["W3"]) * (z1 > 0)'),
    ("first bias gradient summed over units", 'g["b1"] = dz1.sum(axis=0)', 'g["b1"] = dz1.sum(axis=1).sum() * np.ones(N_HID) / N_HID'),
    ("biases laid out before weights", '("W1", (N_HID, N_IN)), ("b1", (N_HID,))', '("b1", (N_HID,)), ("W1", (N_HID, N_IN))'),
    ("weights laid out in x out", '("W1", (N_HID, N_IN))', '("W1", (N_IN, N_HID))'),
]

PINS = [pins.test_param_count, pins.test_parameter_layout, pins.test_gradient_matches_finite_differences,
        pins.test_closed_forms]


def _load(text):
    mod = types.ModuleType("mlp_ref_mutant")
    exec(compile(text, "mlp_ref_mutant.py", "exec"), mod.__dict__)
    return mod


def _all_pins_pass(mod, monkeypatch):
    monkeypatch.setattr(pins, "M", mod)
    try:
        for pin in PINS:
            pin()
    except Exception:  # noqa: BLE001  (a failing or crashing pin catches the mutant)
        return False
    finally:
        monkeypatch.undo()
    return True


@pytest.fixture(scope="module")
def source():
    with open(SRC) as fh:
        return fh.read()


def test_unmodified_reference_passes(source, monkeypatch):
    assert _all_pins_pass(_load(source), monkeypatch)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(source, monkeypatch, name, old, new):
    assert source.count(old) == 1, old
    assert not _all_pins_pass(_load(source.replace(old, new)), monkeypatch), name
