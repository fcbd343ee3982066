"""The oracle's pair-removal and multi-scale variants against facts fixed
by the paper and by geometry (CPU only)."""
import pytest

import oracle
import pins_variants


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


@pytest.mark.parametrize("pin", pins_variants.VARIANT_PINS, ids=lambda f: f.__name__)
def test_variant_pin(orc, pin):
    pin(orc)


def test_rejects_bad_method_arguments(orc):
    import numpy as np
    d = np.ones((8, 8), dtype=np.float32)
    for method, scales in ((3, 0), (-1, 0), ("pair_removal", 2), ("multiscale", 0),
                           ("four_pair", 5)):
        with pytest.raises(ValueError):
            orc.variant_f32(d, 100.0, 100.0, 3.5, 3.5, 1, "rel", 4.0, method=method,
                            scales=scales)
