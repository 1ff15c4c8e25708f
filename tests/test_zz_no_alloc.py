"""The selection entry point that allocates nothing (oed_greedy_noalloc): its workspaces live in the
library's static device array, its kernels are those of oed_create + oed_greedy, so its picks and
gains must equal a handle's bit for bit.  Two calls in a row, the second on a smaller problem
(the array keeps the first call's contents), for every precision."""
import ctypes

import numpy as np
import pytest
import torch

from oed_inputs import make_K

DEV = "cuda:0"

# (N_s, N_t, n_m, seed, budget, delay, K dtype): a larger problem, then a smaller one
CALLS = [(40, 32, 2500, 501, 12, 4, torch.float64), (23, 24, 900, 502, 7, 3, torch.float32)]


def _noalloc(K, N_s, N_t, s2, B, prec, delay):
    from paper_2604_08812_amd import oed_greedy_noalloc
    idx = torch.full((B,), -1, dtype=torch.int32, device=DEV)
    gain = torch.full((B,), float("nan"), dtype=torch.float64, device=DEV)
    st = torch.full((2,), -1, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    oed_greedy_noalloc(K, N_s, N_t, s2, B, idx, gain, st, precision=prec, delay=delay)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return idx.cpu().numpy(), gain.cpu().numpy(), st.cpu().numpy(), free0, free1


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed_f32", "mixed_bf16x3"])
def test_noalloc_equals_handle_twice(prec):
    from paper_2604_08812_amd import Selector
    for q, (N_s, N_t, n_m, seed, B, delay, kdt) in enumerate(CALLS):
        K, s2 = make_K(N_s, N_t, n_m, seed)
        Kd = K.to(DEV).to(kdt)
        print(f"noalloc {prec} call {q}: N_s={N_s} N_t={N_t} B={B} delay={delay} K {kdt}", flush=True)
        idx, gain, st, free0, free1 = _noalloc(Kd, N_s, N_t, s2, B, prec, delay)
        with Selector(Kd, N_s, N_t, s2, precision=prec, delay=delay) as sel:
            i1, g1 = sel.greedy(B)
        assert list(st) == [0, B]
        assert list(idx) == list(i1), (q, idx, i1)
        np.testing.assert_array_equal(gain, g1)
        if q > 0:   # the module (and its static array) is loaded by the first call
            assert free1 >= free0, (free0, free1)


def test_noalloc_rejects_what_it_cannot_hold():
    """Host-side checks before any HIP call (no GPU needed): sizes beyond the static array and
    block sizes beyond the register kernels are OED_E_UNSUPPORTED with a message, bad arguments
    OED_E_ARG."""
    from paper_2604_08812_amd import library
    from paper_2604_08812_amd.oed import OED_NOALLOC_MAX_BYTES
    L = library()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first
    err = ctypes.create_string_buffer(256)

    def call(N_s, N_t, prec=0, delay=4, budget=1, ld=None, s2=1.0, dtype=0):
        ld = N_s * N_t if ld is None else ld
        return L.oed_greedy_noalloc(fake, dtype, ld, N_s, N_t, s2, prec, delay, budget, None, fake, fake, fake,
                                    err, len(err))

    assert call(600, 128, prec=1) == 6 and b"bytes of scratch" in err.value
    assert str(OED_NOALLOC_MAX_BYTES).encode() in err.value
    assert call(256, 64) == 6          # FP64 R alone: 256*257/2 * 64^2 * 8 bytes > 64 MiB
    assert call(4, 160) == 6 and b"N_t" in err.value
    assert call(4, 16, ld=63) == 1
    assert call(4, 16, s2=0.0) == 1
    assert call(4, 16, s2=float("nan")) == 1
    assert call(4, 16, prec=7) == 1
    assert call(4, 16, delay=13) == 1
    assert call(4, 16, budget=5) == 1
    assert call(4, 16, dtype=3) == 1
    assert L.oed_greedy_noalloc(None, 0, 64, 4, 16, 1.0, 0, 4, 1, None, fake, fake, fake, err, len(err)) == 1
    assert L.oed_greedy_noalloc(fake, 0, 64, 4, 16, 1.0, 0, 4, 1, None, None, fake, fake, err, len(err)) == 1
    assert L.oed_greedy_noalloc(fake, 0, 64, 4, 16, 1.0, 0, 4, 1, None, fake, fake, None, None, 0) == 1
