"""nse_nonlinear_adjoint_noalloc (static scratch, no allocation) against
nse_nonlinear_adjoint (the same kernels on allocated intermediates), through the
C ABI: two calls in a row on one device, the second with a smaller input, each
equal to the allocating entry point; a context beyond the scratch is rejected."""
import math
import os

import numpy as np
import pytest
import torch

import nse_inputs as I
import paper_1009_3308_amd as pkg

pytestmark = pytest.mark.gpu
OMEGA = 2.0 * math.pi


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1009_3308_amd import build
        build.build()
    torch.cuda.set_device(0)


def _pair(N, nlat, index):
    print(f"case: no-alloc adjoint N={N} nlat={nlat}", flush=True)
    s = pkg.Sphere([(N, nlat, 1e-5)], omega=OMEGA, dt=1e-3)
    a = pkg.to_device(I.flat_spectrum(N, 40 + index))
    nb = pkg.to_device(I.cotangent(N, 40 + index))
    out = s.new_state()
    s.nonlinear_adjoint_noalloc(a, nb, out)
    got = out.cpu().numpy()
    ref = s.nonlinear_adjoint(a, nb).cpu().numpy()
    s.close()
    return got, ref


def test_noalloc_adjoint_two_calls_second_smaller():
    # T255 on its default grid (the largest member the scratch holds), then a
    # smaller member whose intermediates sit over the first call's contents
    for i, (N, nlat) in enumerate([(255, 0), (63, 100)]):
        got, ref = _pair(N, nlat, i)
        assert np.array_equal(got, ref), N
        assert np.abs(ref).max() > 0


def test_noalloc_adjoint_rejects_beyond_scratch():
    s = pkg.Sphere([(511, 0, 1e-5)], omega=OMEGA, dt=1e-3)
    a, out = s.new_state(), s.new_state()
    with pytest.raises(pkg.NseError) as ei:
        s.nonlinear_adjoint_noalloc(a, a.clone(), out)
    assert ei.value.status == pkg.NSE_ERR_ARG
    assert "static scratch" in str(ei.value)
    s.close()
