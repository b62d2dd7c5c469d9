"""The allocation-free entry point, mickey_generate_rowmajor_noalloc, called through the C
ABI, against the allocating one (mickey_generate_rowmajor) on the same inputs: two calls
in a row, each smaller than the one before, bit for bit, and the states continuing alike."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1909_04750_amd import mickey

pytestmark = pytest.mark.gpu


def inputs(seed, n):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 256, (n, 10), dtype=np.uint8)
    ivs = rng.integers(0, 256, (n, 10), dtype=np.uint8)
    ivb = rng.integers(0, 81, n, dtype=np.uint8)
    return [torch.from_numpy(a).cuda() for a in (keys, ivs, ivb)]


def test_noalloc_equals_allocating_entry_point_twice():
    lib = mickey.load_library()
    # 1,088,000 instances: 864-clock chunks, so the transposes see tiles of 27 clock blocks
    # and rows that start at word 0, 27, 54, 81 and 108 (aligned and unaligned stores);
    # 2^20 + 320 instances: the snapshot takes 25 MiB of the array, leaving 896-clock chunks;
    # each call's output (instances x clocks) is smaller than the one before (the last one
    # has 8192-clock chunks)
    for n, nbits, seed in ((1088000, 4096, 3), ((1 << 20) + 320, 4 * 1024 + 96, 1), (3000, 8192 + 64, 2)):
        k, v, b = inputs(seed, n)
        ref = mickey.Mickey(k, v, b)
        new = mickey.Mickey(k, v, b)
        want_u, want_f = ref.generate_rowmajor(nbits)
        got_u = torch.zeros((n, nbits // 32), dtype=torch.int32, device="cuda")
        got_f = torch.zeros((n, nbits // 32), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        rc = lib.mickey_generate_rowmajor_noalloc(new._h, nbits, ctypes.c_void_p(got_u.data_ptr()),
                                                  ctypes.c_void_p(got_f.data_ptr()))
        assert rc == mickey.OK, lib.mickey_last_error_message()
        new.sync()
        assert torch.equal(got_u, want_u) and torch.equal(got_f.view(torch.int32), want_f.view(torch.int32)), n
        assert new.bits_generated == ref.bits_generated == nbits
        # both states stand at the same clock
        a = ref.generate(64, mickey.ROWMAJOR_U32)
        c = new.generate(64, mickey.ROWMAJOR_U32)
        torch.cuda.synchronize()
        assert torch.equal(a, c), n
        ref.close()
        new.close()


def test_noalloc_rejects_what_does_not_fit():
    lib = mickey.load_library()
    k, v, b = inputs(3, 64)
    m = mickey.Mickey(k, v, b)
    out = torch.zeros(64 * 4, dtype=torch.int32, device="cuda")
    assert lib.mickey_generate_rowmajor_noalloc(m._h, 33, ctypes.c_void_p(out.data_ptr()), None) == mickey.EINVAL
    assert lib.mickey_generate_rowmajor_noalloc(m._h, 32, None, None) == mickey.EINVAL
    m.close()
    n = 9 << 20  # 200 + 64 planes of 1.125 MiB exceed the 256 MiB array
    k, v, _ = inputs(4, 1)
    big = mickey.Mickey(k.repeat(n, 1), v.repeat(n, 1))
    assert lib.mickey_generate_rowmajor_noalloc(big._h, 32, ctypes.c_void_p(out.data_ptr()), None) == mickey.EINVAL
    assert big.bits_generated == 0
    big.close()
