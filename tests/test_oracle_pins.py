"""The oracle against its pins (see tests/pins.py for what fixes each one)."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=[p.__name__ for p in pins.ALL_PINS])
def test_pin(orc, pin):
    pin(orc)


def test_argument_errors(orc):
    import numpy as np
    A = np.eye(3, dtype=np.complex128)
    y = np.ones(3, dtype=np.complex128)
    for bad in (dict(tol=0.0), dict(tol=float("nan")), dict(tol=-1.0),
                dict(maxit=-1)):
        with pytest.raises(ValueError):
            orc.bicgstab(A, y, **bad)
        with pytest.raises(ValueError):
            orc.cgnr(A, y, **bad)
