"""CPU checks of the C-ABI library: it loads without a GPU and exports every function
declared in include/mickey.h (no compute calls here)."""
import ctypes
import os
import re

import pytest

from paper_1909_04750_amd import build, mickey

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("mickey.h", "grain.h", "aes.h", "mickey128.h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names += re.findall(r"\b((?:mickey128|mickey|grain|aes_ctr)_\w+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(build.LIB_PATH):
        build.build_library()
    return mickey.load_library()


def test_header_declares_binding_symbols():
    assert set(declared_functions()) == set(mickey.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(build.LIB_PATH)
    for name in declared_functions():
        assert hasattr(raw, name), name


def test_host_only_queries(lib):
    assert mickey.plane_pitch(1) == 8
    assert mickey.plane_pitch(64) == 8
    assert mickey.plane_pitch(65) == 16
    assert mickey.plane_pitch(1 << 22) == (1 << 22) // 8
    assert mickey.ops_per_clock() == 328
    assert mickey.grain_ops_per_clock() == 36
    assert lib.grain_plane_pitch(65) == 16
    assert lib.aes_ctr_plane_pitch(65) == 16
    assert mickey.aes_ops_per_block() == 9 * 16 * 94 + 9 * 4 * 96 + 80


def test_null_state_is_rejected_without_gpu(lib):
    assert lib.mickey_generate(None, 32, None, 0) == mickey.EINVAL
    assert lib.mickey_last_error() == mickey.EINVAL
    assert b"NULL" in lib.mickey_last_error_message()
    assert lib.mickey_set_word_bits(None, 32) == mickey.EINVAL
    assert lib.mickey_set_schedule(None, mickey.SCHED_SPLIT) == mickey.EINVAL
    assert lib.mickey_set_transpose(None, mickey.TRANSPOSE_STAGED) == mickey.EINVAL
    assert lib.mickey_server_set_kernel(None, 0, 0) == mickey.EINVAL
    assert lib.mickey_num_instances(None) == 0
    lib.mickey_free(None)  # NULL-safe
    assert lib.grain_generate(None, 32, None, 0) == mickey.EINVAL
    assert lib.grain_init(None, None, 4, None) is None
    assert lib.mickey_last_error() == mickey.EINVAL
    assert lib.grain_num_instances(None) == 0
    lib.grain_free(None)
    assert lib.aes_ctr_generate(None, 128, None, 0) == mickey.EINVAL
    assert lib.aes_ctr_init(None, None, 4, None) is None
    lib.aes_ctr_free(None)


def test_chunk_record_layout_matches_binding(tmp_path):
    """The binding reads mickey_chunk records as a numpy structured array: the C struct
    must have the same field offsets and size (compiled here with the host C compiler)."""
    import numpy as np
    import subprocess
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "mickey.h"\n'
                   "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(mickey_chunk),"
                   " offsetof(mickey_chunk, request), offsetof(mickey_chunk, handle), offsetof(mickey_chunk, offset),"
                   " offsetof(mickey_chunk, words), offsetof(mickey_chunk, out), offsetof(mickey_chunk, last));"
                   "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    dt = np.dtype(mickey.Server.CHUNK_DTYPE)
    assert got == [dt.itemsize] + [dt.fields[f][1] for f in dt.names]


def test_headline_kernel_code_hash_is_found():
    """The traffic record is keyed by the headline kernel's machine code: the hash must be
    found in the built library, and differ between kernels."""
    from paper_1909_04750_amd import codeobj
    from paper_1909_04750_amd.build import LIB_PATH
    objs = codeobj.device_code_objects(LIB_PATH)
    assert len(objs) >= 5  # one per HIP source
    h1 = codeobj.kernel_code_hash(LIB_PATH, "_ZN12_GLOBAL__N_120gen_bitsliced_kernelILi1EEEvPjjjmS1_")
    h2 = codeobj.kernel_code_hash(LIB_PATH, "_ZN12_GLOBAL__N_120gen_bitsliced_kernelILi2EEEvPjjjmS1_")
    assert h1 and h2 and h1 != h2 and len(h1) == 16
    assert codeobj.kernel_code_hash(LIB_PATH, "no_such_kernel") is None


def test_request_record_layout_matches_binding(tmp_path):
    """mickey_req as the binding builds it (numpy structured array)."""
    import numpy as np
    import subprocess
    src = tmp_path / "req.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "mickey.h"\n'
                   "int main(void){printf(\"%zu %zu %zu %zu %zu\\n\", sizeof(mickey_req),"
                   " offsetof(mickey_req, instance), offsetof(mickey_req, nbits), offsetof(mickey_req, out),"
                   " offsetof(mickey_req, layout));return 0;}\n")
    exe = tmp_path / "req"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    dt = np.dtype(mickey.REQ_DTYPE)
    assert got == [dt.itemsize] + [dt.fields[f][1] for f in ("instance", "nbits", "out", "layout")]


def test_new_entry_points_validate_without_gpu(lib):
    assert lib.mickey_debug_fail_launch(-1) == mickey.EINVAL
    assert lib.mickey_debug_fail_launch(0) == mickey.OK
    assert lib.mickey_instance_bits(None, 0) == (1 << 64) - 1
    assert lib.mickey_last_error() == mickey.EINVAL
    assert lib.mickey_state_host_bytes(None) == 0
    assert lib.mickey_state_export_host(None, None, 0) == mickey.EINVAL
    assert lib.mickey_state_import_host(None, None, 0) == mickey.EINVAL
    assert lib.mickey_generate_batch(None, None, 0) == mickey.EINVAL
