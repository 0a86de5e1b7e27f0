"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/ptd.h, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ptd.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", src)
    skip = {"if", "defined", "sizeof"}
    return sorted({n for n in names if n not in skip and (n.startswith("ptd_") or n.startswith("pauli_"))})


@pytest.fixture(scope="module")
def lib():
    from paper_2403_11644_amd import _native

    return _native.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert "pauli_decompose" in names and "pauli_reconstruct" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    for st in (0, -1, -2, -3, -4, -5, -99):
        assert lib.ptd_status_str(st)
    assert lib.ptd_build_arch() == b"gfx950"


def test_workspace_sizes(lib):
    # single-pass and two-pass schedules need none; the single-launch schedule
    # (n = 11..15) needs its queue and group counters
    for n in (1, 8, 10, 16):
        for dt in (0, 1):
            assert lib.ptd_workspace_bytes(n, dt, 0, 0) == 0
    # queue words + one counter per group of the narrowest group width
    assert lib.ptd_workspace_bytes(14, 0, 0, 0) == 4 * (32 + (1 << 12))
    assert lib.ptd_workspace_bytes(14, 1, 0, 0) == 4 * (32 + (1 << 11))
    assert lib.ptd_workspace_bytes(15, 0, 0, 0) == 0
    assert lib.ptd_workspace_bytes(14, 0, 1 << 1, 0) == 0  # structured
    assert lib.ptd_workspace_bytes(13, 0, 1, 0) > 0  # Hermitian
    # reconstruction: one launch with counters for n = 11..14, none otherwise
    for n in (1, 10, 15, 16):
        assert lib.ptd_reconstruct_workspace_bytes(n, 0, 0) == 0
    for n in (11, 14):
        for dt in (0, 1):
            assert lib.ptd_reconstruct_workspace_bytes(n, dt, 0) == lib.ptd_workspace_bytes(n, dt, 0, 0)
    assert lib.ptd_reconstruct_workspace_bytes(12, 0, 1 | (1 << 6)) > 0  # Hermitian adjoint
    assert lib.ptd_reconstruct_workspace_bytes(12, 0, 1 << 1) == 0  # not a reconstruct flag
    assert lib.ptd_reconstruct_workspace_bytes(0, 0, 0) == 0


def test_nonempty_counts_match_bruteforce(lib, oracle_mod):
    from paper_2403_11644_amd import api

    for n, s in [(3, 1), (5, 1), (6, 2), (6, 3), (7, 5), (8, 8), (9, 7), (10, 8)]:
        got = api.nonempty_x(n, "banded", s)
        assert got == oracle_mod.nonempty_x_bruteforce(n, s)
        assert len(got) * (1 << n) == oracle_mod.band_term_bound(n, s)
    assert api.nonempty_x(6, "diagonal") == [0]
    assert api.nonempty_x(6, "antidiagonal") == [63]
    assert lib.ptd_num_nonempty_x(6, (1 << 8) | (1 << 1), 0) == -1  # anti-diagonal and diagonal
    assert api.num_nonempty_x(14, "banded", 8) == 96
    assert api.num_nonempty_x(14, "banded", 1) == 15
    assert api.num_nonempty_x(5) == 32


# fake, far-apart "device" addresses: validation must reject before touching them
FAKE_A, FAKE_C, FAKE_W = 1 << 40, 1 << 42, 1 << 44


def _dec(lib, n=4, dt=0, flags=0, s=0, A=FAKE_A, lda=16, C=FAKE_C, ws=None, wsb=0):
    return lib.pauli_decompose(n, dt, flags, s, ctypes.c_void_p(A), lda, ctypes.c_void_p(C),
                               ctypes.c_void_p(ws) if ws else None, wsb, None)


def test_decompose_argument_errors(lib):
    EINVAL, EUNSUP = -1, -3
    # fake non-null "device" pointers: validation must reject before touching them
    assert _dec(lib, n=0) == EINVAL
    assert _dec(lib, n=17, lda=1 << 17) == EINVAL
    assert _dec(lib, dt=2) == EINVAL
    assert _dec(lib, A=0) == EINVAL
    assert _dec(lib, C=0) == EINVAL
    assert _dec(lib, lda=15) == EINVAL
    assert _dec(lib, flags=1 << 12) == EINVAL
    assert _dec(lib, flags=(1 << 1) | (1 << 2), s=1) == EINVAL  # diagonal + banded
    assert _dec(lib, flags=(1 << 2), s=0) == EINVAL  # banded needs s >= 1
    assert _dec(lib, flags=(1 << 2), s=16) == EINVAL  # s < 2^n
    assert _dec(lib, flags=(1 << 3)) == EINVAL  # bands-in without structure
    assert _dec(lib, flags=(1 << 4)) == EINVAL  # compact without structure
    assert _dec(lib, flags=(1 << 6) | (1 << 1)) == EINVAL  # unscaled traces: dense input only
    assert _dec(lib, flags=(1 << 6) | (1 << 5), dt=1) == EINVAL
    assert _dec(lib, flags=(1 << 6) | (1 << 9)) == EINVAL
    assert _dec(lib, flags=(1 << 8) | (1 << 2), s=1) == EINVAL  # anti-diagonal + banded
    assert _dec(lib, flags=(1 << 8) | (1 << 5), dt=1) == -3  # compensated structured: unsupported
    assert _dec(lib, flags=(1 << 5), dt=0) == EUNSUP  # compensated is complex64 only
    assert _dec(lib, A=5, C=5) == EINVAL  # in place is not allowed
    ENOSPC = -2
    assert _dec(lib, n=12, lda=4096, ws=0, wsb=0) == ENOSPC  # single-launch schedule needs counters


def test_decompose_overlap_errors(lib):
    """A, coeff and the workspace must be disjoint byte ranges, not just
    different pointers: the one-launch schedule keeps partial results in
    coeff while it still reads A."""
    EINVAL = -1
    a = FAKE_A
    n = 12
    N = 1 << n
    wsb = lib.ptd_workspace_bytes(n, 0, 0, 0)
    assert wsb > 0
    # coeff starts inside the last row of A (16-byte complex128 elements)
    assert _dec(lib, n=n, lda=N, A=a, C=a + (N * N - 1) * 16, ws=FAKE_W, wsb=wsb) == EINVAL
    # A starts inside coeff
    assert _dec(lib, n=n, lda=N, A=a + 16, C=a, ws=FAKE_W, wsb=wsb) == EINVAL
    # a padded pitch widens the span of A
    assert _dec(lib, n=n, lda=2 * N, A=a, C=a + N * N * 16, ws=FAKE_W, wsb=wsb) == EINVAL
    # the workspace inside A, or inside coeff
    assert _dec(lib, n=n, lda=N, A=a, C=FAKE_C, ws=a + 4096, wsb=wsb) == EINVAL
    assert _dec(lib, n=n, lda=N, A=a, C=FAKE_C, ws=FAKE_C + 64, wsb=wsb) == EINVAL
    # real (Hermitian) output: coeff starting 8 bytes before the end of A
    assert _dec(lib, n=3, lda=8, flags=1, A=a, C=a + 64 * 16 - 8) == EINVAL
    # compact band output: only the nonempty rows count
    rows = lib.ptd_num_nonempty_x(6, 1 << 2, 1)
    assert _dec(lib, n=6, lda=64, flags=(1 << 2) | (1 << 4), s=1, A=a, C=a - rows * 64 * 16 + 16) == EINVAL


def test_reconstruct_overlap_errors(lib):
    EINVAL = -1
    n, N = 12, 1 << 12
    wsb = lib.ptd_reconstruct_workspace_bytes(n, 0, 0)

    def rec(C, A, ws):
        return lib.pauli_reconstruct(n, 0, 0, ctypes.c_void_p(C), ctypes.c_void_p(A), N, ctypes.c_void_p(ws), wsb,
                                     None)

    assert rec(FAKE_C, FAKE_C + 16, FAKE_W) == EINVAL
    assert rec(FAKE_C, FAKE_A, FAKE_A + 1024) == EINVAL


def test_workspace_status_arguments(lib):
    """A call that needs no workspace never waits: status is OK without a
    GPU call; a non-empty but too small workspace is an argument error."""
    assert lib.ptd_workspace_status(None, 0, None) == 0
    assert lib.ptd_workspace_status(None, 256, None) == -1
    assert lib.ptd_workspace_status(ctypes.c_void_p(FAKE_W), 64, None) == -1


def test_reconstruct_argument_errors(lib):
    EINVAL = -1

    def rec(n=4, dt=0, flags=0, C=FAKE_C, A=FAKE_A, lda=16):
        return lib.pauli_reconstruct(n, dt, flags, ctypes.c_void_p(C), ctypes.c_void_p(A), lda, None, 0, None)

    assert rec(n=0) == EINVAL
    assert rec(C=0) == EINVAL
    assert rec(A=0) == EINVAL
    assert rec(lda=8) == EINVAL
    assert rec(flags=1 << 1) == EINVAL
    assert rec(dt=3) == EINVAL
    assert rec(C=5, A=5) == EINVAL  # coefficients and matrix must differ
    ENOSPC = -2
    assert rec(n=12, lda=4096) == ENOSPC  # the single-launch schedule needs its counters


def test_nonempty_x_errors(lib):
    buf = np.zeros(4, dtype=np.uint32)
    assert lib.ptd_nonempty_x(4, 1 << 2, 0, ctypes.c_void_p(buf.ctypes.data)) == -1
    assert lib.ptd_nonempty_x(4, 1 << 2, 1, None) == -1
    assert lib.ptd_num_nonempty_x(0, 0, 0) == -1


def test_labels():
    from paper_2403_11644_amd import labels

    assert labels.label(1, 3, 2) == "ZY"
    for n in (1, 3, 5):
        for x in range(1 << n):
            for z in range(0, 1 << n, 3):
                assert labels.index(labels.label(x, z, n)) == (x, z)
    with pytest.raises(ValueError):
        labels.index("XQ")


def test_tuning_registry(lib):
    cfg, la = ctypes.c_int(), ctypes.c_int()
    lib.ptd_clear_tuning()
    assert lib.ptd_get_tuning(14, 0, 0, ctypes.byref(cfg), ctypes.byref(la)) == 0
    assert lib.ptd_set_tuning(14, 0, 0, 22, 4) == 0
    assert lib.ptd_get_tuning(14, 0, 0, ctypes.byref(cfg), ctypes.byref(la)) == 1
    assert (cfg.value, la.value) == (22, 4)
    assert lib.ptd_get_tuning(14, 0, 1, ctypes.byref(cfg), ctypes.byref(la)) == 0  # Hermitian is separate
    # single-pass sizes tune the group plan: 0..3 for complex64, 0..1 for complex128
    assert lib.ptd_set_tuning(10, 0, 0, 22, 4) == -1
    assert lib.ptd_set_tuning(10, 0, 0, 2, 0) == -1  # radix 32 is complex64 only
    assert lib.ptd_set_tuning(10, 1, 1, 3, 0) == 0
    assert lib.ptd_get_tuning(10, 1, 1, ctypes.byref(cfg), ctypes.byref(la)) == 1
    assert (cfg.value, la.value) == (3, 0)
    assert lib.ptd_get_tuning(10, 1, 0, ctypes.byref(cfg), ctypes.byref(la)) == 0  # default plan
    assert cfg.value == 2  # radix-32 rounds at complex64 n = 10
    assert lib.ptd_get_tuning(9, 0, 0, ctypes.byref(cfg), ctypes.byref(la)) == 0
    assert cfg.value == 0
    assert lib.ptd_set_tuning(14, 0, 0, 99, 4) == -1
    assert lib.ptd_set_tuning(14, 0, 0, 22, 0) == -1
    assert lib.ptd_set_tuning(15, 0, 0, 1, 2) == -1  # complex128 n=15 runs the two-pass schedule
    # a setting must name a shape (bits 0-1); cache-policy bits alone are rejected
    for bad in (4, 8, 12, 16, 28):
        assert lib.ptd_set_tuning(14, 0, 0, bad, 4) == -1
    assert lib.ptd_set_tuning(15, 1, 0, 2, 4) == -1  # n = 15 is built with shape 1 only
    assert lib.ptd_set_tuning(15, 1, 0, 3, 4) == -1
    assert lib.ptd_set_tuning(15, 1, 0, 29, 4) == 0
    lib.ptd_clear_tuning()
    assert lib.ptd_get_tuning(14, 0, 0, ctypes.byref(cfg), ctypes.byref(la)) == 0


def test_batched_argument_errors(lib):
    ns = np.array([3, 11], dtype=np.int32)
    offs = np.zeros(2, dtype=np.int64)
    P = ctypes.c_void_p
    assert lib.ptd_batched_workspace_bytes(2, 0, P(ns.ctypes.data)) == 0  # n = 11 is too large
    ns[1] = 4
    assert lib.ptd_batched_workspace_bytes(2, 0, P(ns.ctypes.data)) > 0
    args = (P(ns.ctypes.data), P(offs.ctypes.data), P(offs.ctypes.data), P(1), P(2))
    assert lib.pauli_decompose_batched(0, 0, 0, *args, None, 0, None) == -1
    assert lib.pauli_decompose_batched(2, 0, 0, *args, None, 0, None) == -2  # no workspace
    assert lib.pauli_decompose_batched(2, 0, 1 << 6, *args, P(3), 1 << 20, None) == -1  # adjoint: reconstruct only
    plan = ctypes.c_void_p()
    assert lib.ptd_batch_plan_create(2, 0, 1 << 6, *args, ctypes.byref(plan)) == -1
    assert lib.ptd_batch_plan_launch(None, None) == -1
    lib.ptd_batch_plan_destroy(None)


def test_pad_to_power_of_two_arguments(lib):
    """Zero padding (Sec. II-A) runs in the library (ptd_zero_pad): a CPU
    tensor is refused, a power-of-two square passes through untouched, and
    the entry point validates sizes and overlap before any HIP call."""
    import torch

    from paper_2403_11644_amd import api

    A8 = torch.zeros((8, 8), dtype=torch.complex128)
    assert api.pad_to_power_of_two(A8) is A8
    with pytest.raises(ValueError):
        api.pad_to_power_of_two(torch.zeros((3, 5), dtype=torch.complex128))
    zp = lib.ptd_zero_pad
    src, dst = ctypes.c_void_p(FAKE_A), ctypes.c_void_p(FAKE_C)
    assert zp(2, src, 5, 3, 5, dst, 3, None) == -1  # dtype
    assert zp(0, None, 5, 3, 5, dst, 3, None) == -1
    assert zp(0, src, 4, 3, 5, dst, 3, None) == -1  # pitch < cols
    assert zp(0, src, 5, 9, 5, dst, 3, None) == -1  # rows > 2^n
    assert zp(0, src, 5, 3, 0, dst, 3, None) == -1
    assert zp(0, src, 5, 3, 5, dst, 0, None) == -1
    assert zp(0, src, 5, 3, 5, ctypes.c_void_p(FAKE_A + 16), 3, None) == -1  # overlap


def test_empty_batch():
    """An empty list of matrices decomposes to an empty list, before any
    device call; the C entry points reject count < 1."""
    from paper_2403_11644_amd import api

    assert api.decompose_batched([]) == []


def test_combination_argument_errors(lib):
    """Sec. IV-B combinations: every bad argument is refused on the host,
    before any device call (bogus addresses never reach a kernel)."""
    EINVAL = -1
    big, far = 1 << 40, 1 << 41  # distinct, far-apart fake device addresses
    bd = lambda k=3, m=2, dt=0, flags=0, b=big, o=far: lib.ptd_block_diagonal(k, m, dt, flags, b, o, None)
    assert bd(k=0) == EINVAL
    assert bd(m=0) == EINVAL
    assert bd(m=6) == EINVAL
    assert bd(k=12, m=5) == EINVAL  # k + m <= 16
    assert bd(dt=2) == EINVAL
    assert bd(flags=1) == EINVAL  # only PTD_COMPACT
    assert bd(b=0) == EINVAL
    assert bd(o=0) == EINVAL
    assert bd(b=big, o=big + 64) == EINVAL  # output overlaps the blocks
    assert bd(o=far + 8) == EINVAL  # output not 16-byte aligned
    ds = lambda n=3, dt=0, flags=0, a=big, b=big + (1 << 20), o=far: lib.ptd_direct_sum(n, dt, flags, a, b, o, None)
    assert ds(n=0) == EINVAL
    assert ds(n=16) == EINVAL  # the result has n + 1 qubits
    assert ds(flags=2) == EINVAL
    assert ds(a=0) == EINVAL
    assert ds(o=big + 16) == EINVAL
    assert ds(o=big + (1 << 20) + 8) == EINVAL
    ha = lambda n=3, dt=1, flags=0, c=big, o=far: lib.ptd_hermitian_augment(n, dt, flags, c, o, None)
    assert ha(n=0) == EINVAL
    assert ha(n=16) == EINVAL
    assert ha(dt=5) == EINVAL
    assert ha(flags=1) == EINVAL
    assert ha(c=0) == EINVAL
    assert ha(o=big) == EINVAL
    assert ha(o=far + 4) == EINVAL
    lc = lambda n=3, dt=0, a=big, b=big + (1 << 20), o=far: lib.ptd_linear_combination(n, dt, 1.0, 0.5, a, b, o,
                                                                                        None)
    assert lc(n=0) == EINVAL
    assert lc(n=17) == EINVAL
    assert lc(dt=2) == EINVAL
    assert lc(a=0) == EINVAL
    assert lc(o=0) == EINVAL
    assert lc(o=big + 16) == EINVAL  # a shifted view of c_a


def test_row_pitch_of_a_single_row():
    """A one-row band array (diagonal / anti-diagonal input) made with a new
    axis has stride 0 on it; its pitch is taken as the row length."""
    import numpy as np
    import torch

    from paper_2403_11644_amd import api

    v = torch.from_numpy(np.arange(8.0)[None, :])
    assert v.stride(0) in (0, 8)
    assert api._rows(v, "v") == 8
    assert api._rows(torch.zeros(3, 8), "m") == 8
    assert api._rows(torch.zeros(8, 16)[:, :8], "m") == 16


def test_lcu_argument_errors(lib):
    EINVAL, ENOSPC = -1, -2
    big, far, ws = 1 << 40, 1 << 41, 1 << 42
    lam = ctypes.c_double()
    wsb = lib.ptd_reduce_workspace_bytes()
    f = lambda n=3, dt=0, flags=0, c=big, o=far, lp=ctypes.byref(lam), w=ws, wb=wsb: lib.ptd_lcu_amplitudes(
        n, dt, flags, c, o, lp, w, wb, None)
    assert f(n=0) == EINVAL
    assert f(n=17) == EINVAL
    assert f(dt=4) == EINVAL
    assert f(flags=2) == EINVAL  # only PTD_HERMITIAN
    assert f(c=0) == EINVAL
    assert f(o=0) == EINVAL
    assert f(lp=None) == EINVAL
    assert f(o=big) == EINVAL  # in place is not allowed
    assert f(w=0) == ENOSPC
    assert f(wb=wsb - 8) == ENOSPC


def test_toeplitz_argument_errors(lib):
    """Matrix-free input: the sizes without a kernel (complex128 at n = 15,
    n = 16) and the structure flags are refused on the host."""
    from paper_2403_11644_amd import api

    EUNSUP = -3
    big, far = 1 << 40, 1 << 41
    dec = lambda n, dt, flags: lib.pauli_decompose(n, dt, flags, 0, big, 0, far, None, 0, None)
    assert dec(15, api.C128, api.TOEPLITZ) == EUNSUP
    assert dec(15, api.C128, api.PURE_STATE | api.HERMITIAN) == EUNSUP
    assert dec(16, api.C64, api.TOEPLITZ) == EUNSUP
    assert dec(16, api.C64, api.PURE_STATE) == EUNSUP
    assert dec(12, api.C64, api.TOEPLITZ | api.DIAGONAL) == EUNSUP
    assert dec(12, api.C64, api.TOEPLITZ | api.COMPENSATED) == EUNSUP
    assert dec(3, api.C64, api.TOEPLITZ | api.COMPACT) == -1  # compact needs a structure
    # low-rank factor: rank in 1..32, row pitch >= rank, one matrix-free kind per call
    lr = lambda n, flags, s, lda: lib.pauli_decompose(n, api.C128, flags, s, big, lda, far, None, 0, None)
    assert lr(8, api.LOW_RANK, 0, 4) == -1
    assert lr(8, api.LOW_RANK, 33, 40) == -1
    assert lr(8, api.LOW_RANK, 4, 3) == -1
    assert lr(8, api.LOW_RANK, 4, (1 << 40) + 1) == -1
    assert lr(8, api.LOW_RANK | api.PURE_STATE, 1, 1) == -1
    assert lr(8, api.LOW_RANK | api.TOEPLITZ, 1, 1) == -1
    assert lr(8, api.LOW_RANK | api.DIAGONAL, 2, 2) == EUNSUP
    assert lr(15, api.LOW_RANK, 2, 2) == EUNSUP
    assert lr(16, api.LOW_RANK, 2, 2) == EUNSUP
    # n >= 11: the factor's transpose is staged in the workspace
    assert lib.ptd_workspace_bytes(14, api.C128, api.LOW_RANK, 2) == 2 * (1 << 14) * 16
    assert lib.ptd_workspace_bytes(15, api.C64, api.LOW_RANK | api.HERMITIAN, 32) == 32 * (1 << 15) * 8
    assert lib.ptd_workspace_bytes(10, api.C128, api.LOW_RANK, 2) == 0
    assert lr(12, api.LOW_RANK, 2, 2) == -2  # no workspace given


def test_to_dict():
    """{label: coefficient} view of dense and compact arrays."""
    import numpy as np

    from paper_2403_11644_amd import labels

    c = np.zeros((4, 4), dtype=np.complex128)
    c[0, 0] = 0.5           # II
    c[1, 3] = -0.25j        # Y on qubit 0, Z on qubit 1: 'ZY'
    c[3, 0] = 1e-20         # below the tolerance
    d = labels.to_dict(c, tol=1e-12)
    assert d == {"II": 0.5, labels.label(1, 3, 2): -0.25j}
    assert labels.label(1, 3, 2) == "ZY"
    # compact rows with their X-patterns; real (Hermitian) arrays give floats
    r = np.array([[0.0, 2.0], [0.0, -1.0]])
    assert labels.to_dict(r, xs=[0, 1]) == {"Z": 2.0, "Y": -1.0}
    with pytest.raises(ValueError):
        labels.to_dict(np.zeros((1, 4)))  # compact without xs


def test_bandwidth_probe_arguments(lib):
    """The bandwidth reference hook validates its shape bits before any HIP call."""
    bw = lib.ptd_debug_bandwidth
    a, c = ctypes.c_void_p(FAKE_A), ctypes.c_void_p(FAKE_C)
    assert bw(0, a, c, 4096 + 8, None) == -1  # not a multiple of 16 bytes
    assert bw(0, None, c, 4096, None) == -1  # copy needs a source
    assert bw(2 | (3 << 8), None, c, 4096, None) == -1  # 2048-thread workgroups
    assert bw(2 | (2 << 8) | (2 << 10), None, c, 4096, None) == -1  # 1024 threads x 4 per CU
    assert bw(1 << 7, a, c, 4096, None) == -1  # unused bit
    assert bw(3, None, c, 4096, None) == -1  # write-back probe: 64 KiB granules
    assert bw(3 | (1 << 4), None, c, 65536, None) == -1  # write-back probe takes no other bits
    assert bw(3, None, None, 65536, None) == -1
    assert bw(3, None, c, 2 << 30, None) == -1  # at most 1 GiB


def test_autotune_report_arguments(lib):
    f, g, h, k = ctypes.c_float(), ctypes.c_float(), ctypes.c_float(), ctypes.c_int()
    lib.ptd_clear_tuning()
    assert lib.ptd_autotune_report(12, 0, 0, ctypes.byref(f), ctypes.byref(g), ctypes.byref(h), ctypes.byref(k)) == 0
    assert lib.ptd_autotune_report(12, 0, 2, ctypes.byref(f), ctypes.byref(g), ctypes.byref(h), ctypes.byref(k)) == -1
    assert lib.ptd_autotune_report(12, 0, 0, None, ctypes.byref(g), ctypes.byref(h), ctypes.byref(k)) == -1


def test_csr_argument_errors(lib):
    """Compressed-row input: argument and overlap errors come back before
    any HIP call (fake device addresses are never dereferenced)."""
    EINVAL, ENOSPC = -1, -2
    n = 6
    N = 1 << n
    wsb = lib.ptd_sparse_workspace_bytes(n)
    assert wsb == 4 * N + 256
    rp, ci, va, xs, out, ws = (ctypes.c_void_p(FAKE_A + k * (1 << 24)) for k in range(6))
    cnt = ctypes.c_int()
    # nonempty list: bad n, negative nnz, missing arrays, short workspace
    assert lib.ptd_csr_nonempty_x(0, 4, rp, ci, xs, ctypes.byref(cnt), ws, wsb, None) == EINVAL
    assert lib.ptd_csr_nonempty_x(n, -1, rp, ci, xs, ctypes.byref(cnt), ws, wsb, None) == EINVAL
    assert lib.ptd_csr_nonempty_x(n, 4, None, ci, xs, ctypes.byref(cnt), ws, wsb, None) == EINVAL
    assert lib.ptd_csr_nonempty_x(n, 4, rp, None, xs, ctypes.byref(cnt), ws, wsb, None) == EINVAL
    assert lib.ptd_csr_nonempty_x(n, 4, rp, ci, None, ctypes.byref(cnt), ws, wsb, None) == EINVAL
    assert lib.ptd_csr_nonempty_x(n, 4, rp, ci, xs, None, ws, wsb, None) == EINVAL
    assert lib.ptd_csr_nonempty_x(n, 4, rp, ci, xs, ctypes.byref(cnt), ws, wsb - 1, None) == ENOSPC
    assert lib.ptd_csr_nonempty_x(n, 4, rp, ci, xs, ctypes.byref(cnt), None, wsb, None) == ENOSPC
    # the workspace over row_ptr (2^n + 1 int64 values) or the list over col_idx
    assert lib.ptd_csr_nonempty_x(n, 4, rp, ci, xs, ctypes.byref(cnt), ctypes.c_void_p(FAKE_A + 8 * N), wsb,
                                  None) == EINVAL
    assert lib.ptd_csr_nonempty_x(n, 4, rp, ci, ctypes.c_void_p(FAKE_A + (1 << 24) + 12), ctypes.byref(cnt), ws, wsb,
                                  None) == EINVAL

    def dec(flags=0, nnz=4, dt=0, rp=rp, ci=ci, va=va, xs=xs, count=2, out=out, ws=ws, wsb=wsb):
        return lib.pauli_decompose_csr(n, dt, flags, nnz, rp, ci, va, xs, count, out, ws, wsb, None)

    assert dec(dt=7) == EINVAL
    assert dec(flags=1) == EINVAL  # only PTD_COMPACT
    assert dec(nnz=-1) == EINVAL
    assert dec(rp=None) == EINVAL and dec(ci=None) == EINVAL and dec(va=None) == EINVAL
    assert dec(count=-1) == EINVAL and dec(count=N + 1) == EINVAL and dec(xs=None) == EINVAL
    assert dec(out=None) == EINVAL
    assert dec(wsb=wsb - 1) == ENOSPC
    # the output over the values, over row_ptr's last value, or over the
    # workspace; the workspace over the list
    assert dec(out=ctypes.c_void_p(FAKE_A + 2 * (1 << 24) + 48)) == EINVAL
    assert dec(out=ctypes.c_void_p(FAKE_A + 8 * N)) == EINVAL
    assert dec(out=ctypes.c_void_p(FAKE_A + 5 * (1 << 24) - N * N * 16 + 16)) == EINVAL
    assert dec(ws=ctypes.c_void_p(FAKE_A + 3 * (1 << 24) + 4)) == EINVAL
    # compact output: count rows of it, ending 16 bytes into the values
    assert dec(flags=1 << 2, out=ctypes.c_void_p(FAKE_A + 2 * (1 << 24) - 2 * N * 16 + 16)) == EINVAL


def test_describe_tuning(lib):
    """The single-launch settings in the schedule's terms: threads, low WHT
    stages per phase-1 item (the stage split), X-patterns per group (T)."""
    from paper_2403_11644_amd import api, tuning

    assert tuning.describe(14, api.C128, False, 1) == {"threads": 1024, "phase1_bits": 10, "phase2_bits": 4,
                                                       "group_patterns": 8}
    assert tuning.describe(14, api.C128, False, 2) == {"threads": 512, "phase1_bits": 9, "phase2_bits": 5,
                                                       "group_patterns": 8}
    assert tuning.describe(13, api.C64, True, 3 | 4 | 8) == {"threads": 512, "phase1_bits": 10, "phase2_bits": 3,
                                                             "group_patterns": 8}
    assert tuning.describe(15, api.C64, False, 1)["group_patterns"] == 16
    # the default setting is one of the built shapes at every point
    for n in range(11, 16):
        for dt in (api.C128, api.C64):
            for herm in (False, True):
                if n == 15 and (dt == api.C128 or herm):
                    continue
                d = tuning.describe(n, dt, herm, 0)
                assert d["threads"] in (512, 1024) and d["phase1_bits"] in (9, 10)
    th, kap, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    args = (ctypes.byref(th), ctypes.byref(kap), ctypes.byref(t))
    assert lib.ptd_describe_tuning(15, api.C128, 0, 1, *args) == -1  # not built
    assert lib.ptd_describe_tuning(15, api.C64, 0, 2, *args) == -1  # shape 2 stops at n = 14
    assert lib.ptd_describe_tuning(10, api.C64, 0, 1, *args) == -1  # the group kernel's plans
    assert lib.ptd_describe_tuning(14, api.C64, 0, 32, *args) == -1
    assert lib.ptd_describe_tuning(14, api.C64, 2, 1, *args) == -1
    assert lib.ptd_describe_tuning(14, api.C64, 0, 1, None, ctypes.byref(kap), ctypes.byref(t)) == -1
