"""CPU checks of the test-side rounding helpers."""
import numpy as np

from tests import rounding_model as RM


def test_relu_undecided_rows_flags_only_near_zero_preactivations():
    # two hidden layers of width 2 and an output row; record 0 puts the second
    # layer's first unit at exactly 0 (1 - 1), record 1 at 1e-9 of its terms'
    # magnitude, record 2 keeps every unit far from zero
    w1 = np.eye(2)
    w2 = np.array([[1.0, -1.0], [1.0, 1.0]])
    wo = np.ones((1, 2))
    x = np.array([[1.0, 1.0], [1.0, 1.0 - 1e-9], [2.0, 1.0]])
    got = RM.relu_undecided_rows([w1, w2, wo], x)
    assert got.tolist() == [True, True, False]
    # the output layer is linear: a zero output decides no mask
    assert not RM.relu_undecided_rows([w1, np.array([[1.0, -1.0]])], np.array([[1.0, 1.0]]))[0]
