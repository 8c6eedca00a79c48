"""The library's own check of its memory layouts (qtx_check_layouts): the
regions that the sweep, decimation and Newton kernels and the
no-allocation plan carve out of one allocation stay aligned, inside it and
disjoint, for every block size, slab count and precision.  The kernels take
their offsets from the same layout function, so this is a host-side bounds
check of what they address; it needs no device."""
import ctypes
import re

from paper_1903_00548_amd import _lib


def test_layouts_are_disjoint_and_in_bounds():
    lib = _lib.load()
    buf = ctypes.create_string_buffer(1024)
    rc = lib.qtx_check_layouts(buf, len(buf))
    msg = buf.value.decode()
    assert rc == 0, msg
    m = re.fullmatch(r"ok: (\d+) sweep, (\d+) decimation, (\d+) no-allocation layouts", msg)
    assert m, msg
    n_sweep, n_dec, n_plan = map(int, m.groups())
    # 6 block sizes x 7 slab counts x 2 launch sizes x (fp64, mixed, its fp64 re-solve, density matrix)
    assert n_sweep == 6 * 7 * 2 * 4
    assert n_dec == 6
    assert n_plan > 100          # most of the 6 x 4 x 4 x 4 problems fit the scratch


def test_null_message_is_accepted():
    assert _lib.load().qtx_check_layouts(None, 0) == 0
