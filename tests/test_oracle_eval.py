"""The evaluation oracle (angle images, MSE, plane fit) against closed forms
(CPU only)."""
import pytest

import pins_eval


@pytest.mark.parametrize("pin", pins_eval.EVAL_PINS, ids=lambda f: f.__name__)
def test_eval_pin(pin):
    pin()
