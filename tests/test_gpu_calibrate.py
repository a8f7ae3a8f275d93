"""The roofline calibration entry point: both kinds return a plausible
positive rate for one MI355X-class device, and other kinds are rejected."""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_calibrate_rates():
    from paper_2408_00384_amd import (CAL_LDS, CAL_VALU, CLIFF_EINVAL, CliffError, Context,
                                      cliff_calibrate)
    ctx = Context(0)
    lds = cliff_calibrate(ctx.handle, CAL_LDS)
    valu = cliff_calibrate(ctx.handle, CAL_VALU)
    assert math.isfinite(lds) and 1e12 < lds < 1e15        # bytes/s
    assert math.isfinite(valu) and 1e12 < valu < 1e15      # lane ops/s
    with pytest.raises(CliffError) as e:
        cliff_calibrate(ctx.handle, 2)
    assert e.value.code == CLIFF_EINVAL
    ctx.close()
