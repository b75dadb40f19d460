"""C-ABI checks that need no GPU: the library loads, exports every function
include/hydro.h declares, and rejects bad arguments on the host (before any
device call) with HYDRO_EINVAL and a message."""
import ctypes as C

import pytest

from paper_2507_09337_amd import hydro as H
from paper_2507_09337_amd import inputs as I

FAKE_ARENA = C.c_void_p(0x10000)  # never dereferenced: validation fails first


@pytest.mark.parametrize("lang,std", [("c", "-std=c99"), ("c++", "-std=c++11")])
def test_header_is_plain_c(lang, std):
    """include/hydro.h needs no HIP or C++ header: it compiles on its own as
    C99 and as C++ (plain pointers, sizes and opaque handles only)."""
    import shutil
    import subprocess

    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no gcc")
    r = subprocess.run([cc, "-fsyntax-only", "-Wall", "-Werror", "-x", lang, std, H.HEADER], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stderr


def test_library_exports_every_declared_function():
    names = H.declared_functions()
    assert len(names) >= 15
    L = H.lib()
    for n in names:
        assert hasattr(L, n), n


def _create(mesh, ndim=None, arena_len=None, arena=FAKE_ARENA):
    descs = H.descs_from_mesh(mesh)
    h = C.c_void_p()
    rc = H.lib().hydro_mesh_create(descs, len(descs), mesh.ndim if ndim is None else ndim, arena,
                                   mesh.arena_len if arena_len is None else arena_len, None, C.byref(h))
    return rc, H.lib().hydro_last_error().decode()


def good():
    return I.block_grid((2, 2, 1), (16, 16, 4), (0, 0, 0), (1, 1, 1), "periodic", 3)


@pytest.mark.parametrize(
    "mutate,needle",
    [
        (lambda m: m.n.__setitem__((0, 0), 12), "multiples of 8"),
        (lambda m: m.kind.__setitem__((1, 2), 7), "face kind"),
        (lambda m: m.nbr.__setitem__((2, 1), 99), "out of range"),
        (lambda m: m.offset.__setitem__(1, 3), "overlap"),
        (lambda m: m.offset.__setitem__(3, 10**9), "outside the arena"),
        (lambda m: m.dx.__setitem__((0, 1), -1.0), "dx"),
        (lambda m: m.dx.__setitem__((0, 2), float("nan")), "dx"),
        (lambda m: m.n.__setitem__((0, 2), 1), "n[2]"),
    ],
)
def test_bad_descriptor_rejected_on_host(mutate, needle):
    m = good()
    arena_len = m.arena_len
    mutate(m)
    rc, msg = _create(m, arena_len=arena_len)
    assert rc == H.EINVAL and needle in msg, msg


def test_valid_mesh_without_gpu_fails_loudly_or_succeeds():
    """A valid descriptor passes host validation; with no GPU the call must
    then fail with EDEVICE (never silently succeed on the CPU)."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, msg = _create(good())
    assert rc == H.EDEVICE and msg


def test_tangential_mismatch_rejected():
    m = I.independent_blocks([16, 16], 3)
    m.kind[0, 0] = I.NBR
    m.nbr[0, 0] = 1
    m.n[1] = (16, 16, 8)  # tangential z extent differs
    m.offset[1] = 5 * 16 ** 3
    rc, msg = _create(m)
    assert rc == H.EINVAL and "tangential" in msg


def test_2d_requires_unit_z():
    m = I.block_grid((2, 1, 1), (16, 16, 1), (0, 0, 0), (1, 1, 1), "outflow", 2)
    m.n[0, 2] = 2
    rc, msg = _create(m, ndim=2)
    assert rc == H.EINVAL and "2D" in msg


def test_bad_ndim_null_arena_and_null_handles():
    m = good()
    assert _create(m, ndim=4)[0] == H.EINVAL
    assert _create(m, arena=C.c_void_p(None))[0] == H.EINVAL
    assert _create(m, arena_len=0)[0] == H.EINVAL
    L = H.lib()
    out = C.c_void_p()
    ids = (C.c_int32 * 1)(0)
    assert L.hydro_packet_create(None, ids, 1, 0, C.byref(out)) == H.EINVAL
    assert L.hydro_packet_advance(None, 1e-3, 1.4) == H.EINVAL
    assert L.hydro_batch_run(None, 1, 0.4, 1.4, None) == H.EINVAL
    assert L.hydro_batch_create(None, 0, C.byref(out)) == H.EINVAL
    assert L.hydro_mesh_destroy(None) == H.EINVAL
    assert L.hydro_last_error()  # a message is set


def test_every_handle_call_rejects_a_null_handle():
    """Each call that takes a packet, batch or stream handle returns EINVAL
    with a message for a null handle, before any device call."""
    L = H.lib()
    d = C.c_double()
    i = C.c_int32()
    cfg = (C.c_int32 * 64)()
    calls = {
        "hydro_packet_reduce_dt": (None, 1.4, 0.4, C.byref(d)),
        "hydro_packet_destroy": (None,),
        "hydro_batch_advance_plain": (None, 1e-3, 1.4),
        "hydro_batch_run_timed": (None, 1, 0.4, 1.4, None, C.byref(d)),
        "hydro_batch_time_kernels": (None, 1, 0.4, 1.4, C.byref(d)),
        "hydro_batch_set_tiling": (None, 16, 16, 0),
        "hydro_batch_set_launch": (None, 0, 1),
        "hydro_batch_set_occupancy": (None, 3),
        "hydro_batch_autotune": (None, 1.4, 1),
        "hydro_batch_get_config": (None, cfg, 16, C.byref(i)),
        "hydro_batch_destroy": (None,),
        "hydro_stream_run": (None, 1, 0.4, 1.4, None),
        "hydro_stream_set_cpu_share": (None, 1, 1),
        "hydro_stream_set_unit_bytes": (None, 1 << 20),
        "hydro_stream_destroy": (None,),
    }
    for name, args in calls.items():
        L.hydro_last_error()
        assert getattr(L, name)(*args) == H.EINVAL, name
        assert L.hydro_last_error(), name


def test_empty_inputs_rejected_on_host():
    """No blocks, no packets, no block ids: EINVAL with a message, before any
    device call."""
    m = good()
    descs = H.descs_from_mesh(m)
    L = H.lib()
    h = C.c_void_p()
    assert L.hydro_mesh_create(descs, 0, 3, FAKE_ARENA, m.arena_len, None, C.byref(h)) == H.EINVAL
    assert "nblocks" in L.hydro_last_error().decode()
    ids = (C.c_int32 * 1)(0)
    assert L.hydro_packet_create(None, ids, 0, 0, C.byref(h)) == H.EINVAL
    st = (C.c_int32 * 1)(0)
    assert L.hydro_stream_create(descs, len(descs), 3, FAKE_ARENA, m.arena_len, st, 0, 0, 2, C.byref(h)) == H.EINVAL
    assert L.hydro_step_static(descs, 0, 3, FAKE_ARENA, m.arena_len, 0, 1e-3, 1.4, None) == H.EINVAL


class _Host:
    """Stand-in host arena (never dereferenced: validation fails first)."""

    def __init__(self, n):
        self.n = n

    def data_ptr(self):
        return 0x10000

    def numel(self):
        return self.n


@pytest.mark.parametrize("case", ["ranges", "gap", "open"])
def test_host_stream_rejects_bad_packets_on_host(case):
    m = I.independent_blocks([8, 16, 8, 8], 3)
    packets = [range(0, 2), range(2, 4)]
    if case == "ranges":
        packets = [range(0, 2), range(2, 3)]  # block 3 in no packet
    elif case == "gap":
        m.offset[1] += 8  # block 1 no longer follows block 0
    else:
        m.kind[0, 1] = I.NBR
        m.nbr[0, 1] = 3  # links outside packet 0
    with pytest.raises(H.HydroError) as e:
        H.HostStream(m, _Host(m.arena_len + 64), packets)
    assert e.value.code == H.EINVAL


@pytest.mark.parametrize("prec", [2, 0x1001, 0x1100, 0x1400, 0x300, 0x701, 0xC01, 0x101 | 0x2000, -1])
def test_bad_precision_codes_rejected_on_host(prec):
    m = I.independent_blocks([8, 8], 3)
    with pytest.raises(H.HydroError) as e:
        H.HostStream(m, _Host(m.arena_len), [range(0, 1), range(1, 2)], prec)
    assert e.value.code == H.EINVAL and "precision" in str(e.value)


@pytest.mark.parametrize("prec", [H.FP64 | H.EINFELDT, H.FP32_FP64 | H.EINFELDT, H.FP64 | H.PVRS,
                                  H.FP32_FP64 | H.PVRS, H.FP64 | H.CONSERVED, H.FP32_FP64 | H.CONSERVED | H.PVRS,
                                  H.FP64 | H.CHARACTERISTIC, H.FP32_FP64 | H.CHARACTERISTIC | H.EINFELDT,
                                  H.FP64 | H.GAS_RADIATION])
def test_method_variants_pass_host_validation(prec):
    """A valid code with method-variant flags gets past every host check; with
    no GPU the first device call then fails loudly."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("host-only check (the stand-in arena is not real memory)")
    m = I.independent_blocks([8, 8], 3)
    try:
        H.HostStream(m, _Host(m.arena_len), [range(0, 1), range(1, 2)], prec).close()
    except H.HydroError as e:
        assert e.code in (H.EDEVICE, H.ENOMEM), str(e)


def test_extent_and_count_limits_rejected_on_host():
    m = I.block_grid((1, 1, 1), (16392, 8, 2), (0, 0, 0), (1, 1, 1), "periodic", 3)
    rc, msg = _create(m)
    assert rc == H.EINVAL and "16384" in msg, msg
    descs = H.descs_from_mesh(good())
    h = C.c_void_p()
    assert H.lib().hydro_mesh_create(descs, 0, 3, FAKE_ARENA, 100, None, C.byref(h)) == H.EINVAL


def test_static_step_rejects_on_host():
    """The allocation-free step checks sizes and arguments on the host before
    any device work: a mesh beyond the fixed scratch, too many blocks, a bad
    descriptor, dt or precision are EINVAL with a message."""
    lib = H.lib()

    def call(m, prec=H.FP64, dt=1e-3, gamma=1.4):
        descs = H.descs_from_mesh(m)
        rc = lib.hydro_step_static(descs, len(descs), m.ndim, FAKE_ARENA, m.arena_len, prec, dt, gamma, None)
        return rc, lib.hydro_last_error().decode()

    big = I.block_grid((8, 8, 8), (16, 16, 16), (0, 0, 0), (1, 1, 1), "periodic", 3)  # 80 MiB of stage state
    rc, msg = call(big)
    assert rc == H.EINVAL and "scratch" in msg, msg
    rc, msg = call(I.independent_blocks([8] * 4097, 3))
    assert rc == H.EINVAL and "4096" in msg, msg
    m = good()
    m.n[0, 0] = 12
    rc, msg = call(m)
    assert rc == H.EINVAL and "multiples of 8" in msg, msg
    rc, msg = call(good(), dt=float("nan"))
    assert rc == H.EINVAL and "dt" in msg, msg
    rc, msg = call(good(), gamma=1.0)
    assert rc == H.EINVAL and "gamma" in msg, msg
    rc, msg = call(good(), prec=7)
    assert rc == H.EINVAL and "precision" in msg, msg
