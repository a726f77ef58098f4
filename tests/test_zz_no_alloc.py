"""The allocation-free interpolation entry point (tdslda_interp2d_noalloc)
against the allocating one (tdslda_interp2d) through the C ABI: two calls
in a row on the same GPU (the second with a smaller source and target
lattice, so the shared coefficient array holds the first call's larger
contents), then a source lattice beyond the fixed array's limit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    torch.cuda.set_device(0)


def _field(nx, ny, seed):
    # a smooth periodic field plus seeded noise (band-limited or not does
    # not matter here: both entry points compute the same sums)
    g = synth.rng(seed)
    x = np.arange(nx)[:, None] / nx
    y = np.arange(ny)[None, :] / ny
    return np.cos(2 * np.pi * x) * np.sin(4 * np.pi * y) + 0.1 * g.standard_normal((nx, ny))


def test_noalloc_equals_allocating_entry_point():
    from paper_2602_08982_amd import tdslda as T
    T.load_library()
    stream = torch.cuda.current_stream()
    # (source shape, spacing), (target shape, spacing) over one box per case
    cases = [((24, 20), (1.0, 1.2), (32, 30), (0.75, 0.8)),
             ((8, 6), (2.0, 2.0), (12, 10), (4.0 / 3.0, 1.2))]
    for k, (s1, d1, s2, d2) in enumerate(cases):
        f = _field(*s1, seed=40 + k)
        ref = T.interp2d(f, d1, s2, d2)
        f_dev = torch.from_numpy(f).to("cuda")
        out_dev = torch.full(s2, np.nan, dtype=torch.float64, device="cuda")
        T.interp2d_noalloc(f_dev, d1, out_dev, d2, stream.cuda_stream)
        torch.cuda.synchronize()
        got = out_dev.cpu().numpy()
        # same kernels on the same inputs: identical to the last bit
        assert np.array_equal(got, ref), (k, float(np.abs(got - ref).max()))


def test_noalloc_rejects_a_source_beyond_the_fixed_array():
    from paper_2602_08982_amd import tdslda as T
    T.load_library()
    f_dev = torch.zeros((258, 256), dtype=torch.float64, device="cuda")  # 66048 > 65536 points
    out_dev = torch.zeros((258, 256), dtype=torch.float64, device="cuda")
    with pytest.raises(T.TdsldaError) as e:
        T.interp2d_noalloc(f_dev, (1.0, 1.0), out_dev, (1.0, 1.0))
    assert e.value.status == T.EINVAL
    # a box mismatch is rejected the same way, before any launch
    small = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(T.TdsldaError):
        T.interp2d_noalloc(small, (1.0, 1.0), small, (2.0, 1.0))
