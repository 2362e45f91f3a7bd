"""hmps_svd_probe_noalloc (the allocation-free variant of hmps_svd_probe,
its intermediates in the library's file-scope device array) against the
existing entry point on the same theta': the kept rank, the singular values
and both factors must be identical (the two share every kernel of the
update's SVD).  Two calls in a row on one device, the second on a smaller
theta', and a third on the in-LDS path, so that each call runs on what the
previous one left in the shared array; plus the size limit."""
import ctypes as C

import numpy as np
import pytest

from paper_1910_09142_amd import hmps

pytestmark = pytest.mark.gpu


def theta_of(seed, m, n):
    """Seeded theta' with a graded spectrum (Haar factors, exp decay)."""
    rng = np.random.Generator(np.random.Philox(seed))
    k = min(m, n)
    u, _ = np.linalg.qr(rng.standard_normal((m, k)))
    v, _ = np.linalg.qr(rng.standard_normal((n, k)))
    s = np.exp(-np.arange(k) / 30.0)
    t = (u * s) @ v.T
    return t / np.linalg.norm(t)


def probe_existing(theta, chi_max, cutoff):
    chi_l, chi_r = theta.shape[0] // 3, theta.shape[1] // 3
    ctx = hmps.Context(1, 2, 128, 1)   # the variant's capacity: chi <= 128
    out = ctx.hmps_svd_probe(theta, chi_max, cutoff)
    ctx.hmps_destroy()
    return out


def probe_noalloc(theta, chi_max, cutoff):
    import torch
    lib = hmps.load()
    m, n = theta.shape
    chi_l, chi_r = m // 3, n // 3
    kmax = min(m, n)
    dev = torch.device("cuda:0")
    th = torch.from_numpy(np.ascontiguousarray(theta)).to(dev)
    sig = torch.zeros(kmax, dtype=torch.float64, device=dev)
    left = torch.zeros(3 * chi_l * kmax, dtype=torch.float64, device=dev)
    right = torch.zeros(3 * kmax * chi_r, dtype=torch.float64, device=dev)
    rank = C.c_int32(0)
    stream = torch.cuda.current_stream(dev)
    st = lib.hmps_svd_probe_noalloc(
        0, C.c_void_p(stream.cuda_stream), chi_l, chi_r,
        C.c_void_p(th.data_ptr()), chi_max, cutoff,
        C.c_void_p(sig.data_ptr()), C.byref(rank),
        C.c_void_p(left.data_ptr()), C.c_void_p(right.data_ptr()))
    torch.cuda.synchronize()
    if st:
        raise hmps.HmpsError(st, "hmps_svd_probe_noalloc")
    k = rank.value
    return (sig[:k].cpu().numpy(),
            left[:3 * chi_l * k].cpu().numpy().reshape(3, chi_l, k),
            right[:3 * k * chi_r].cpu().numpy().reshape(3, k, chi_r))


@pytest.mark.parametrize("order", ["large_first"])
def test_noalloc_equals_the_existing_probe(order):
    # 384 x 300 (QR-preconditioned blocked rounds), then 120 x 60 (blocked,
    # fewer blocks), then 24 x 27 (in-LDS): each call reuses the array
    cases = [(1, 384, 300, 100, 1e-10), (2, 120, 60, 40, 1e-12),
             (3, 24, 27, 16, 1e-10)]
    for seed, m, n, chi_max, cut in cases:
        print(f"case: noalloc probe {m}x{n} chi_max={chi_max}", flush=True)
        theta = theta_of(seed, m, n)
        s0, l0, r0 = probe_existing(theta, chi_max, cut)
        s1, l1, r1 = probe_noalloc(theta, chi_max, cut)
        assert s0.shape == s1.shape
        assert np.array_equal(s0, s1)
        assert np.array_equal(l0, l1)
        assert np.array_equal(r0, r1)
        # and against LAPACK (the truncated SVD it computes)
        s = np.linalg.svd(theta, compute_uv=False)
        assert np.abs(s1 - s[:len(s1)]).max() <= 1e-12 * s[0]


def test_noalloc_rejects_sizes_beyond_its_array():
    import torch
    lib = hmps.load()
    dev = torch.device("cuda:0")
    x = torch.zeros(16, dtype=torch.float64, device=dev)
    rank = C.c_int32(0)
    p = C.c_void_p(x.data_ptr())
    # chi_l = 129 > 128
    st = lib.hmps_svd_probe_noalloc(0, None, 129, 4, p, 8, 1e-10, p,
                                    C.byref(rank), p, p)
    assert st == hmps.HMPS_E_INVALID
    st = lib.hmps_svd_probe_noalloc(0, None, 4, 4, None, 8, 1e-10, p,
                                    C.byref(rank), p, p)
    assert st == hmps.HMPS_E_INVALID
