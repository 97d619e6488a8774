"""The allocation-free projection (fft_homog_project_noalloc) against the handle's projection.

Collected last (test_zz_*) on purpose: it must pass after every other GPU test of the process
as well as alone.

Two calls in a row, the second with a smaller input, each compared with fft_homog_debug_project
of a handle of the same descriptor (same launches, the handle's workspace as scratch): the two
differ only in the twiddle tables (device sincospi here, host extended precision there), so the
fields agree to a few units of rounding.  A request beyond the 64 MiB scratch is refused before
any launch.
"""

import numpy as np
import pytest

from helpers import field_err
from paper_2408_03804_amd import binding

pytestmark = pytest.mark.gpu


def reference(shape, kin, mat, x):
    h = binding.FFTHomog(shape, kin, mat, 2, tangent=x.shape[0] > 1)
    return h.debug_project(x).cpu().numpy().reshape(x.shape)


def noalloc(shape, kin, mat, x):
    import torch
    d = binding.make_desc(shape, kin, mat, 2)
    out = torch.full_like(x, float("nan"))
    binding.fft_homog_project_noalloc(d, x, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_two_calls_in_a_row_match_the_handle_projection():
    import torch
    cases = [((24, 20, 18), "finite", "neo_hookean", 2),   # first call: 2 fields of 9 components
             ((9, 7, 5), "small", "linear_elastic", 1)]     # second call: smaller
    for shape, kin, mat, batch in cases:
        c = 9 if kin == "finite" else 6
        x = torch.as_tensor(np.random.default_rng(7).standard_normal((batch, c) + shape)).cuda()
        got = noalloc(shape, kin, mat, x)
        ref = reference(shape, kin, mat, x)
        assert np.all(np.isfinite(got))
        assert field_err(got, ref) < 1e-13, (shape, kin)


def test_2d_and_request_beyond_the_scratch():
    import torch
    shape = (31, 31)
    x = torch.as_tensor(np.random.default_rng(3).standard_normal((1, 3) + shape)).cuda()
    assert field_err(noalloc(shape, "small", "linear_elastic", x), reference(shape, "small", "linear_elastic", x)) < 1e-13
    # axes that take the chirp-z transform (its tables live in the scratch too): x in 2D, outer in 3D
    for shp, kin, mat, c in (((199, 8), "small", "linear_elastic", 3), ((4, 5, 97), "finite", "neo_hookean", 9)):
        xc = torch.as_tensor(np.random.default_rng(5).standard_normal((1, c) + shp)).cuda()
        assert field_err(noalloc(shp, kin, mat, xc), reference(shp, kin, mat, xc)) < 1e-13, shp
    # 128^3 finite strain: a 170 MB half spectrum does not fit the 64 MiB scratch
    big = (128, 128, 128)
    d = binding.make_desc(big, "finite", "neo_hookean", 2)
    xb = torch.empty((1, 9) + big, dtype=torch.float64, device="cuda")
    with pytest.raises(binding.FFTHomogError) as ei:
        binding.fft_homog_project_noalloc(d, xb, torch.empty_like(xb))
    assert ei.value.status == "eworkspace" and "scratch" in str(ei.value)
