"""tdse_dissimilarity_noalloc (the eq. (16) dissimilarity with the library's
fixed per-GPU scratch in place of a workspace) against tdse_dissimilarity
on the same inputs: two calls in a row, the second on a smaller input, so
the second reads a scratch array the first left full of its own partial
sums.  Both entry points run the same kernels with the same plan, so the
results agree bit for bit."""
import ctypes

import pytest
import torch

from paper_2401_07416_amd import tdse

pytestmark = pytest.mark.gpu


def frames_of(K, T, P, dtype, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    f = torch.rand((K, T, P), generator=g, device="cuda", dtype=torch.float64)
    return f.to(dtype).contiguous()


def weights_of(T):
    return torch.full((T,), 1.0 / T, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_matches_workspace_entry_point_twice(dtype):
    cases = [(300, 12, 4099, 11), (70, 5, 333, 12)]   # second call smaller
    for K, T, P, seed in cases:
        print(f"no-alloc dissimilarity {dtype} K={K} T={T} P={P} seed={seed}", flush=True)
        fr = frames_of(K, T, P, dtype, seed)
        w = weights_of(T)
        ref = tdse.dissimilarity(fr, w, 0.04)
        got = tdse.dissimilarity_noalloc(fr, w, 0.04)
        torch.cuda.synchronize()
        assert got.shape == (K, K)
        assert torch.equal(got, ref), (got - ref).abs().max().item()
        assert torch.all(got.diagonal() == 0)


def test_noalloc_with_pairs_in_the_direct_form_twice():
    """FP32 frames with a tight cluster far from trajectory 0, whose pairs go
    through the list of pairs evaluated in the direct form (kept in the same
    scratch), then a smaller input with fewer such pairs: bitwise the
    workspace entry point's result both times."""
    for K, T, P, n, seed in [(260, 6, 1500, 50, 14), (90, 3, 700, 8, 15)]:
        print(f"no-alloc dissimilarity cluster K={K} T={T} P={P} n={n} seed={seed}", flush=True)
        fr = frames_of(K, T, P, torch.float64, seed)
        g = torch.Generator(device="cuda")
        g.manual_seed(seed + 100)
        base = fr[K // 2:K // 2 + 1] + 2.0
        fr[K // 2 - n // 2:K // 2 - n // 2 + n] = base + 1e-6 * torch.randn(
            (n, T, P), generator=g, device="cuda", dtype=torch.float64)
        fr = fr.to(torch.float32).contiguous()
        w = weights_of(T)
        ref = tdse.dissimilarity(fr, w, 0.04)
        got = tdse.dissimilarity_noalloc(fr, w, 0.04)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (got - ref).abs().max().item()
        i = K // 2 - n // 2
        assert 0 < ref[i, i + 1].item() < 1e-4 * ref[0, i].item()


def test_noalloc_rejects_partials_beyond_its_scratch():
    lib = tdse.load()
    nb = ctypes.c_size_t()
    K, T = 2000, 77
    assert lib.tdse_dissimilarity_workspace_size(K, T, ctypes.byref(nb)) == tdse.OK
    assert nb.value > tdse.DISSIM_NOALLOC_MAX_BYTES
    fake = ctypes.c_void_p(256)   # never dereferenced: rejected before any launch
    st = lib.tdse_dissimilarity_noalloc(tdse.F32, fake, K, T, 16384, fake, 0.04, fake, None)
    assert st == tdse.ERR_CAPACITY


def test_noalloc_fits_the_paper_sample():
    """FP32 records of 879 trajectories x 77 frames (the paper's sample of
    section 3.2; 53 MiB of partial sums and 3 MiB of pair list) fit the fixed
    scratch; a short
    pixel row keeps the run cheap, the plan depends on K and T only."""
    K, T, P = 879, 77, 64
    print(f"no-alloc dissimilarity float32 K={K} T={T} P={P}", flush=True)
    fr = frames_of(K, T, P, torch.float32, 13)
    w = weights_of(T)
    ref = tdse.dissimilarity(fr, w, 0.04)
    got = tdse.dissimilarity_noalloc(fr, w, 0.04)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
