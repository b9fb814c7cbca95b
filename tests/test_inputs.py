"""The seeded input generators (shared by both sides; no stepping arithmetic)."""
import numpy as np
import pytest
import torch

from paper_2105_09671_amd import inputs


def test_splitmix64_matches_published_sequence():
    # SplitMix64 started from state 0 (Steele, Lea & Flood 2014; the
    # reference generator's first three outputs)
    z = inputs._mix64(np.arange(1, 4, dtype=np.uint64) * inputs.GOLDEN)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_range_and_moments():
    u = inputs.uniform01(3, 0, 1 << 16)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01 and abs(u.var() - 1 / 12) < 0.005


@pytest.mark.parametrize("shape,seed,stream", [((37, 53), 5, 0), ((8, 16, 9), 6, 3), ((300, 301), 1, 1000)])
def test_chunked_and_torch_fields_are_identical(shape, seed, stream):
    ref = inputs.random_field(shape, seed, stream)
    assert np.array_equal(ref, inputs.random_field(shape, seed, stream, chunk=777))
    assert np.array_equal(ref, inputs.random_field_torch(shape, seed, stream, chunk=1000).numpy())
    f32 = inputs.random_field(shape, seed, stream, dtype=np.float32)
    assert np.array_equal(f32, ref.astype(np.float32))
    t32 = inputs.random_field_torch(shape, seed, stream, dtype=torch.float32).numpy()
    assert np.array_equal(f32, t32)
    assert np.abs(ref).max() <= 0.1
