"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/psm.h, and rejects bad arguments with
PSM_EINVAL before anything is enqueued."""
import ctypes
import os
import re

import pytest

import paper_2303_11811_amd as psm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "psm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psm_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 20
    L = psm.lib()
    for n in names:
        assert hasattr(L, n), n
        assert n in psm._SIGS, f"binding lacks {n}"


def test_workspace_size_scales_with_storage():
    d = [psm.make_desc(64, 48, 40, 0.6, max_particles=10, max_radius=5.0)]
    s64 = psm.psm_workspace_size(d, psm.PSM_FP64)
    s32 = psm.psm_workspace_size(d, psm.PSM_FP32DEV)
    s16 = psm.psm_workspace_size(d, psm.PSM_FP16DEV)
    grid = 2 * 19 * 64 * 48 * 40
    assert s64 - s32 == grid * 4 and s32 - s16 == grid * 2
    assert s64 > grid * 8


@pytest.mark.parametrize("desc,msg", [
    (dict(nx=3, ny=8, nz=8, tau=0.6), "dimension"),
    (dict(nx=8, ny=8, nz=8, tau=0.5), "tau"),
    (dict(nx=8, ny=8, nz=8, tau=float("nan")), "tau"),
    (dict(nx=16, ny=16, nz=16, tau=0.6, max_particles=2, max_radius=0.5), "max_radius"),
    (dict(nx=16, ny=16, nz=16, tau=0.6, max_particles=2, max_radius=7.0), "2*(max_radius+1)+2"),
    (dict(nx=16, ny=16, nz=16, tau=0.6, mapping=7), "mapping"),
    (dict(nx=16, ny=16, nz=16, tau=0.6, mapping=1, subsample_n=0), "subsample_n"),
    (dict(nx=16, ny=16, nz=16, tau=0.6, max_particles=-1), "max_particles"),
])
def test_invalid_descriptors(desc, msg):
    with pytest.raises(psm.PsmError) as e:
        psm.psm_workspace_size([psm.make_desc(**desc)], psm.PSM_FP64)
    assert e.value.code == psm.PSM_EINVAL and msg in str(e.value)


def test_invalid_storage_and_empty():
    with pytest.raises(psm.PsmError):
        psm.psm_workspace_size([psm.make_desc(8, 8, 8, 0.6)], 7)
    out = ctypes.c_size_t(0)
    assert psm.lib().psm_workspace_size(None, 0, 0, ctypes.byref(out)) == psm.PSM_EINVAL


def test_create_rejects_before_touching_the_gpu():
    d = [psm.make_desc(8, 8, 8, 0.6)]
    need = psm.psm_workspace_size(d, psm.PSM_FP64)
    for ws, nbytes, msg in [(0, need, "NULL"), (256 + 8, need, "aligned"), (1 << 20, need - 1, "needs")]:
        with pytest.raises(psm.PsmError) as e:
            psm.psm_create(d, psm.PSM_FP64, 0.0, 0, ws, nbytes)
        assert e.value.code == psm.PSM_EINVAL and msg in str(e.value)
    with pytest.raises(psm.PsmError) as e:
        psm.psm_create(d, psm.PSM_FP16DEV, 3.0, 0, 1 << 20, 1 << 40)
    assert "power of two" in str(e.value)


def test_null_context_calls():
    L = psm.lib()
    assert L.psm_step(None, 1) == psm.PSM_EINVAL
    assert L.psm_destroy(None) == psm.PSM_EINVAL
    assert L.psm_set_graph(None, 1) == psm.PSM_EINVAL
    assert L.psm_get_forces(None, 0, None, None) == psm.PSM_EINVAL
    assert L.psm_integrate(None, 1.0, psm.PSM_VERLET) == psm.PSM_EINVAL
    assert L.psm_run(None, 10, 1.0, psm.PSM_VERLET) == psm.PSM_EINVAL
    assert L.psm_set_dynamics(None, 0, 1.0, None) == psm.PSM_EINVAL
    assert L.psm_get_particles(None, 0, None, None, None) == psm.PSM_EINVAL
    assert L.psm_set_launch(None, 64, 4, 1, 0) == psm.PSM_EINVAL
    assert L.psm_set_drift_check(None, 0, 1e-12) == psm.PSM_EINVAL
    assert L.psm_set_strict_slots(None, 1) == psm.PSM_EINVAL
    assert L.psm_set_force_readback(None, 1) == psm.PSM_EINVAL
    assert "NULL" in psm.psm_last_error() or "ctx" in psm.psm_last_error()


def test_stream_copy_argument_checks():
    L = psm.lib()
    assert L.psm_stream_copy(None, None, 16, None) == psm.PSM_EINVAL
    ms = ctypes.c_double(0)
    assert L.psm_pattern_copy(None, 1, 1, ctypes.byref(ms)) == psm.PSM_EINVAL
    assert L.psm_stream_copy(ctypes.c_void_p(256), ctypes.c_void_p(4096), 15, None) == psm.PSM_EINVAL
    assert L.psm_stream_copy(ctypes.c_void_p(256), ctypes.c_void_p(264), 64, None) == psm.PSM_EINVAL


def test_header_is_plain_c_and_links(tmp_path):
    """include/psm.h compiles as C99 on its own, and a C program calling the
    host-only entry points links against libpsm.so and runs without a GPU."""
    import shutil
    import subprocess

    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "abi.c"
    src.write_text(r'''
#include <stdio.h>
#include "psm.h"
int main(void) {
    psm_box_desc d = {0};
    size_t bytes = 0;
    d.nx = 40; d.ny = 36; d.nz = 30; d.tau = 0.7;
    d.max_particles = 4; d.max_radius = 4.0; d.mapping = PSM_MAP_LINEAR; d.subsample_n = 4;
    d.walls_z = 1; d.face_type[0] = PSM_FACE_VELOCITY; d.face_type[1] = PSM_FACE_PRESSURE;
    d.face_rho[1] = 1.0;
    if (psm_workspace_size(&d, 1, PSM_FP32DEV, &bytes) != PSM_OK || bytes == 0) return 1;
    d.tau = 0.4;
    if (psm_workspace_size(&d, 1, PSM_FP32DEV, &bytes) != PSM_EINVAL) return 2;
    if (psm_step(NULL, 1) != PSM_EINVAL) return 3;
    printf("%zu %s\n", bytes, psm_last_error());
    return 0;
}
''')
    exe = tmp_path / "abi"
    libdir = os.path.dirname(psm.LIB_PATH)
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe), "-L", libdir, "-lpsm", f"-Wl,-rpath,{libdir}"], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, (out.returncode, out.stdout, out.stderr)
    assert "ctx" in out.stdout


def test_row_pitch_padding_in_workspace_size():
    """Rows are padded to whole 64-cell blocks when that adds at most 1/8 to
    the row (nx 57-64 take the grid bytes of nx 64), narrower ones are packed
    (nx 56 takes less). Tile counts agree for these widths at every tile
    width, so the grids are the only difference."""
    def ws(nx):
        return psm.psm_workspace_size([psm.make_desc(nx, 16, 8, 0.6, max_particles=2, max_radius=2.0)],
                                      psm.PSM_FP64)
    assert ws(60) == ws(64) and ws(57) == ws(64)
    grid64 = 2 * 8 * (64 * 16 // 64) * 19 * 64 * 8
    grid56 = 2 * 8 * -(-(56 * 16) // 64) * 19 * 64 * 8
    assert ws(64) - ws(56) == grid64 - grid56


def test_last_error_is_per_thread():
    """Two threads failing in different ways each read back their own error
    text (psm_last_error is thread-local)."""
    import threading

    L = psm.lib()
    bad = {"tau": psm.make_desc(8, 8, 8, 0.4), "dimension": psm.make_desc(3, 8, 8, 0.6)}
    seen = {}
    barrier = threading.Barrier(2)

    def worker(key):
        arr = psm._desc_array([bad[key]])
        out = ctypes.c_size_t(0)
        msgs = []
        for _ in range(200):
            barrier.wait()
            assert L.psm_workspace_size(arr, 1, psm.PSM_FP64, ctypes.byref(out)) == psm.PSM_EINVAL
            barrier.wait()
            msgs.append(psm.psm_last_error())
        seen[key] = msgs

    ts = [threading.Thread(target=worker, args=(k,)) for k in bad]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    for key, msgs in seen.items():
        assert len(msgs) == 200 and all(key in m for m in msgs), (key, set(msgs))


def test_plane_size_limit():
    """In-plane byte offsets are 32-bit signed: a z-plane (rows padded to whole
    64-cell blocks, 19 FP64 values per cell, plus one block) must stay below
    2^31 bytes. 4096 x 3449 cells fit, 4096 x 3450 do not."""
    ok = psm.make_desc(4096, 3449, 4, 0.6)
    assert 4096 * 3449 * 19 * 8 + 64 * 19 * 8 < 2 ** 31 <= 4096 * 3450 * 19 * 8 + 64 * 19 * 8
    assert psm.psm_workspace_size([ok], psm.PSM_FP16DEV) > 0
    with pytest.raises(psm.PsmError) as e:
        psm.psm_workspace_size([psm.make_desc(4096, 3450, 4, 0.6)], psm.PSM_FP16DEV)
    assert e.value.code == psm.PSM_EINVAL and "2^31" in str(e.value)
