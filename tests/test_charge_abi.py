"""The library's charge schedule (host arithmetic, no device work) against
the oracle's, for every model, at the end points and in between."""
import math
import os

import pytest

from oracle import charge_oracle as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2511_10073_amd", "libahr.so")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libahr.so not built")
@pytest.mark.parametrize("model", [Q.GAUSSIAN, Q.EXPONENTIAL, Q.LINEAR, Q.SIGMOID])
def test_schedule_matches_oracle(model):
    import numpy as np
    import paper_2511_10073_amd as A
    f32 = lambda v: float(np.float32(v))
    for t in (0, 1, 37, 60, 150, 240, 299, 300):
        cp = A.charge_params(model=model, t=t, T=300, sigma_factor=0.007, k_factor=1.5)
        ref = Q.schedule(Q.ChargeParams(model=model, t=t, T=300, sigma_factor=f32(0.007), k_factor=f32(1.5),
                                        r0=f32(1e-3), r1=f32(0.9), beta_min=f32(0.1), beta_max=f32(1.0),
                                        alpha0=f32(0.2), alpha1=f32(0.8)))
        got = A.charge_schedule(cp)
        if math.isinf(ref):
            assert math.isinf(got)
        else:
            assert math.isclose(got, ref, rel_tol=1e-15, abs_tol=0), (model, t, got, ref)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libahr.so not built")
def test_charge_params_validated_before_device_work():
    import ctypes
    import paper_2511_10073_amd as A
    lib = A.load()
    v = ctypes.c_double()
    for bad in (A.charge_params(model=7), A.charge_params(t=301, T=300), A.charge_params(T=0),
                A.charge_params(nbx=0), A.charge_params(sigma_factor=0.0),
                A.charge_params(model=A.CHARGE_GAUSSIAN, r0=1.5), A.charge_params(model=A.CHARGE_GAUSSIAN, alpha0=0.9,
                                                                                   alpha1=0.5),
                A.charge_params(model=A.CHARGE_SIGMOID, k_factor=-1.0)):
        assert lib.ahr_charge_schedule(ctypes.byref(bad), ctypes.byref(v)) == A.EINVAL
