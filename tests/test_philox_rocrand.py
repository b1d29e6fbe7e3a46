"""The oracle's Philox4x32-10 against rocRAND's host implementation.

rocRAND creates its host generator only where a HIP device exists, so this
pin runs with the GPU tests.  rocRAND's philox4x32_10 stream for a seed s
starts at counter 0 with key (lo32(s), hi32(s)) and emits the four words of
each block in order; the block counter advances in the first counter word.
"""
import ctypes as C

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

ROCRAND_RNG_PSEUDO_PHILOX4_32_10 = 404


def _rocrand_words(seed, n):
    lib = C.CDLL("/opt/rocm/lib/librocrand.so")
    gen = C.c_void_p()
    assert lib.rocrand_create_generator_host_blocking(C.byref(gen), ROCRAND_RNG_PSEUDO_PHILOX4_32_10) == 0
    try:
        assert lib.rocrand_set_seed(gen, C.c_ulonglong(seed)) == 0
        out = np.zeros(n, dtype=np.uint32)
        assert lib.rocrand_generate(gen, out.ctypes.data_as(C.c_void_p), C.c_size_t(n)) == 0
        return out
    finally:
        lib.rocrand_destroy_generator(gen)


@pytest.mark.parametrize("seed", [0, 1, 0x123456789ABCDEF])
def test_oracle_philox_matches_rocrand_stream(seed):
    n = 64
    ref = _rocrand_words(seed, n)
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    mine = np.concatenate([O.philox([b, 0, 0, 0], key) for b in range(n // 4)])
    assert np.array_equal(mine, ref), (mine[:8], ref[:8])
