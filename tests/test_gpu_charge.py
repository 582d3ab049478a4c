"""GPU parity of the macro charge-density bin integrals (Section VI) through
the C ABI against the FP64 oracle.

Bar (derived from the arithmetic): every per-pair integral is float64 on
both sides (closed forms or quadrature within about 1e-13 of the macro
area), and the device adds them in 2^-28 fixed point, so each bin agrees to
1e-10 relative plus 1e-7 absolute (area units)."""
import math

import numpy as np
import pytest
import torch

from oracle import charge_oracle as Q
from synth import netlist as N

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2511_10073_amd")

MODELS = [Q.GAUSSIAN, Q.EXPONENTIAL, Q.LINEAR, Q.SIGMOID]


def f32(v):
    return float(np.float32(v))


def oracle_params(model, t, T, nbx, nby, sf, kf):
    return Q.ChargeParams(model=model, t=t, T=T, nbx=nbx, nby=nby, sigma_factor=f32(sf), k_factor=f32(kf),
                          r0=f32(1e-3), r1=f32(0.9), beta_min=f32(0.1), beta_max=f32(1.0), alpha0=f32(0.2),
                          alpha1=f32(0.8))


def gpu_mass(nl, model, t, T, nbx, nby, sf=0.005, kf=1.0):
    net = A.Netlist(nl)
    x = torch.as_tensor(nl["g0"]).cuda()
    cp = A.charge_params(model=model, t=t, T=T, nbx=nbx, nby=nby, sigma_factor=sf, k_factor=kf)
    a = A.macro_charge(net, x, cp)
    b = A.macro_charge(net, x, cp)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    return a.cpu().numpy()


def close(got, ref):
    assert np.all(np.abs(got - ref) <= 1e-10 * np.abs(ref) + 1e-7), np.max(np.abs(got - ref))


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("t", [0, 45, 150, 270, 300])
def test_charge_tiny_matches_oracle(model, t):
    nl = N.generate(N.TINY)             # 8 movable macros of 20-60 rows, some across bins and the die edge
    got = gpu_mass(nl, model, t, 300, 8, 8)
    ref = Q.bin_mass(nl, nl["g0"], oracle_params(model, t, 300, 8, 8, 0.005, 1.0))
    close(got, ref)


@pytest.mark.parametrize("model", MODELS)
def test_charge_small_fixed_macros(model):
    nl = N.generate(N.small(5000, 3, ncols=2))     # fixed macros, a non-square bin grid
    got = gpu_mass(nl, model, 100, 300, 12, 7, sf=0.01, kf=2.0)
    ref = Q.bin_mass(nl, nl["g0"], oracle_params(model, 100, 300, 12, 7, 0.01, 2.0))
    close(got, ref)


@pytest.mark.parametrize("model", [Q.GAUSSIAN, Q.EXPONENTIAL])
def test_charge_full_size_large_every_bin(model):
    nl = N.generate(N.LARGE)            # 8,000 fixed macros, 32 x 32 bins
    got = gpu_mass(nl, model, 120, 300, 32, 32)
    ref = Q.bin_mass(nl, nl["g0"], oracle_params(model, 120, 300, 32, 32, 0.005, 1.0))
    close(got, ref)


@pytest.mark.parametrize("model", [Q.LINEAR, Q.SIGMOID])
def test_charge_full_size_large_total(model):
    """Radial models at large-2.2M: rho is the same function of (dx/w, dy/h)
    for every macro, so a macro inside the die carries w h I(k) with I(k) its
    integral over the unit footprint; the few macros crossing the die edge
    are integrated one by one.  The bins' total must equal that sum."""
    nl = N.generate(N.LARGE)
    got = gpu_mass(nl, model, 120, 300, 32, 32)
    cp = oracle_params(model, 120, 300, 32, 32, 0.005, 1.0)
    k = Q.schedule(cp)
    unit = Q.pair_mass(model, k, -0.5, 0.5, -0.5, 0.5, 1.0, 1.0)
    d = nl["die"].astype(np.float64)
    ids = Q.macro_ids(nl)
    pos = nl["g0"][:, :2].astype(np.float32).astype(np.float64)
    size = nl["node_size"].astype(np.float64)
    inside = ((pos[ids, 0] - size[ids, 0] / 2 >= d[0]) & (pos[ids, 0] + size[ids, 0] / 2 <= d[2])
              & (pos[ids, 1] - size[ids, 1] / 2 >= d[1]) & (pos[ids, 1] + size[ids, 1] / 2 <= d[3]))
    total = unit * float((size[ids[inside], 0] * size[ids[inside], 1]).sum())
    edge = ids[~inside]
    if edge.size:
        total += Q.bin_mass(nl, nl["g0"], cp, macros=edge).sum()
    print(f"[charge] model {model}: {inside.sum()} macros inside, {edge.size} on the edge", flush=True)
    assert math.isclose(got.sum(), total, rel_tol=1e-10)
