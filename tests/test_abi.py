"""CPU checks of the C-ABI boundary: the library loads, exports every symbol
include/psl.h declares, and the binding's structs match the header's layout."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psl.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"PSL_API[^;(]*?\b(psl_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("psl_ctx_create", "psl_init_walks", "psl_eval_neighbourhood",
                 "psl_apply_flip", "psl_step_batch", "psl_read_walk"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2107_09801_amd import libpsl
    lib = libpsl.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(libpsl.EXPORTS) == _declared()


def test_struct_layouts_match_header(tmp_path):
    from paper_2107_09801_amd import libpsl
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "psl.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                   ' sizeof(psl_walk_cfg), sizeof(psl_choice), sizeof(psl_walk_state),'
                   ' offsetof(psl_walk_state, t), offsetof(psl_choice, F_min), sizeof(psl_serve_cfg),'
                   ' sizeof(psl_job), sizeof(psl_job_result), sizeof(psl_serve_stats),'
                   ' sizeof(psl_timing)); printf("%zu %zu\\n", sizeof(psl_tune_choice), sizeof(psl_trace_entry)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(libpsl.WalkCfg), ctypes.sizeof(libpsl.Choice),
            ctypes.sizeof(libpsl.WalkState), libpsl.WalkState.t.offset, libpsl.Choice.F_min.offset,
            ctypes.sizeof(libpsl.ServeCfg), ctypes.sizeof(libpsl.Job),
            ctypes.sizeof(libpsl.JobResult), ctypes.sizeof(libpsl.ServeStats),
            ctypes.sizeof(libpsl.Timing), ctypes.sizeof(libpsl.TuneChoice),
            ctypes.sizeof(libpsl.TraceEntry)]
    assert got == want


def test_version_and_shape_without_gpu():
    from paper_2107_09801_amd import libpsl
    assert "gfx950" in libpsl.version()
    lib = libpsl.lib()
    t, k = ctypes.c_uint32(), ctypes.c_uint32()
    # 1024 walks: 16-wavefront blocks of 1024 candidates, one k-split
    assert lib.psl_eval_shape(None, 131071, 131071, 1024, ctypes.byref(t), ctypes.byref(k)) == 0
    assert t.value == 128 and k.value == 1
    # 64 walks at Table 4's N_lmt = 6912: 16-wavefront blocks, items cut to 2^23 updates
    assert lib.psl_eval_shape(None, 131071, 6912, 64, ctypes.byref(t), ctypes.byref(k)) == 0
    assert t.value == 7 and k.value == 16
    assert lib.psl_eval_shape(None, 131071, 6912, (1 << 20) + 1, ctypes.byref(t), ctypes.byref(k)) == libpsl.E_INVAL
    assert lib.psl_eval_shape(None, 16383, 16383, 1, ctypes.byref(t), ctypes.byref(k)) == 0
    assert t.value == 32 and k.value >= 8
    assert lib.psl_eval_shape(None, 1, 1, 1, ctypes.byref(t), ctypes.byref(k)) == libpsl.E_INVAL
    # one long walk: items of at most 2^24 updates (16384 shifts of a
    # 1024-candidate tile), 65536 of them
    assert lib.psl_eval_shape(None, 1048575, 1048575, 1, ctypes.byref(t), ctypes.byref(k)) == 0
    assert t.value == 1024 and k.value == 64
    # short items are not cut further: about 4096 items
    assert lib.psl_eval_shape(None, 1048575, 6912, 1, ctypes.byref(t), ctypes.byref(k)) == 0
    assert t.value == 14 and 4096 <= t.value * k.value < 4200


def test_serve_footprint_without_gpu():
    from paper_2107_09801_amd import libpsl
    a = libpsl.serve_footprint(30001, 256)
    b = libpsl.serve_footprint(30001, 0)
    c = libpsl.serve_footprint(1048575, 0)
    assert 0 < a < b < c
    assert c > 4 * 1048575 * 2           # at least C and C of local_best
    with pytest.raises(libpsl.PslError):
        libpsl.serve_footprint(1, 0)


def test_null_context_is_rejected_without_gpu():
    from paper_2107_09801_amd import libpsl
    lib = libpsl.lib()
    assert lib.psl_sync(None) == libpsl.E_INVAL
    assert lib.psl_step_batch(None, None, 0, 1, 0) == libpsl.E_INVAL
    assert lib.psl_last_error(None) == b"null context"
    out = ctypes.c_void_p()
    # no device here: creation fails cleanly with an error status
    st = lib.psl_ctx_create(0, None, None, 0, ctypes.byref(out))
    if st != libpsl.OK:
        assert st in (libpsl.E_INVAL, libpsl.E_HIP) and not out.value
    else:
        lib.psl_ctx_destroy(out)
        pytest.skip("a device is present")


def test_bench_refuses_more_than_one_gpu():
    # walks run on one GPU: any other count exits with a message and status 2
    # before the device is touched
    import json
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "--gpus must be 1" in msg["error"]
