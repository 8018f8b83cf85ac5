"""C ABI checks that need no GPU: the library loads, exports every function
that include/mm.h declares, and rejects null arguments without touching a
device."""
import ctypes as C
import os
import re

import pytest

import paper_2504_20937_amd as mm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            text = open(os.path.join(inc, f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(mm_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    L = mm.lib()
    names = _declared()
    assert len(names) >= 19
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert missing == []


def test_binding_wraps_every_declared_symbol():
    for n in _declared():
        assert hasattr(mm, n) or n in ("mm_status_string", "mm_last_error"), n


def test_status_strings():
    assert mm.status_name(mm.MM_OK) == "MM_OK"
    assert mm.status_name(mm.MM_ERR_IN_USE) == "MM_ERR_IN_USE"
    assert mm.status_name(-99) == "MM_ERR_UNKNOWN"
    assert mm.mm_version() >= 100


def test_null_arguments_are_rejected_without_a_device():
    L = mm.lib()
    out = C.c_void_p()
    assert L.mm_create_instance(None, C.byref(out)) == mm.MM_ERR_INVALID_ARG
    assert out.value is None  # out-param untouched
    assert "null" in mm.mm_last_error()
    for name in ["mm_destroy_instance", "mm_synchronize", "mm_free", "mm_destroy_view",
                 "mm_render"]:
        assert getattr(L, name)(None) == mm.MM_ERR_INVALID_ARG, name
    assert L.mm_step(None, 0) == mm.MM_ERR_INVALID_ARG
    assert L.mm_step_render(None, 0) == mm.MM_ERR_INVALID_ARG
    assert L.mm_create_view(None, None, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_alloc_linear(None, 16, None, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_profile_begin(None, 4) == mm.MM_ERR_INVALID_ARG
    assert L.mm_profile_every(None, 4) == mm.MM_ERR_INVALID_ARG
    assert L.mm_mark_begin(None, 4) == mm.MM_ERR_INVALID_ARG
    assert L.mm_mark_end(None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_step_render_static(None) == mm.MM_ERR_INVALID_ARG
    n = C.c_uint32(77)
    assert L.mm_mark_read(None, None, C.byref(n)) == mm.MM_ERR_INVALID_ARG
    assert n.value == 77  # out-param untouched
    assert L.mm_prepare_views(None, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_update_views(None, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_set_colour(None, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_set_frame_overlap(None, 1) == mm.MM_ERR_INVALID_ARG
    assert L.mm_flush_frame(None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_create_grid(None, None, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_destroy_grid(None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_grid_render(None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_grid_read_frame(None, None, 0) == mm.MM_ERR_INVALID_ARG
    assert L.mm_create_edges(None, None, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_destroy_edges(None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_edges_render(None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_edges_set_camera(None, None) == mm.MM_ERR_INVALID_ARG


def test_view_desc_layout_matches_header():
    # offsets of the C struct on x86-64: pointer, u64, two enums, 3 u32, pad, u64, f32, i32, f32[16]
    d = mm.mm_view_desc
    assert d.position.offset == 0
    assert d.element_count.offset == 8
    assert d.format.offset == 16 and d.domain.offset == 20
    assert d.width.offset == 24 and d.height.offset == 28 and d.footprint.offset == 32
    assert d.seed.offset == 40
    assert d.amplitude.offset == 48 and d.wrap.offset == 52
    assert d.view_proj.offset == 56
    assert C.sizeof(d) == 120


def test_header_struct_layout_compiles_to_the_same_offsets(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "mm.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu\\n\", offsetof(mm_view_desc, seed),"
        " offsetof(mm_view_desc, amplitude), offsetof(mm_view_desc, wrap),"
        " offsetof(mm_view_desc, view_proj), sizeof(mm_view_desc), sizeof(mm_instance_desc));"
        "return 0;}\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert out == ["40", "48", "52", "56", "120", str(C.sizeof(mm.mm_instance_desc))]


def test_batch_calls_reject_null_arguments_without_a_device():
    L = mm.lib()
    assert L.mm_create_batch(None, None, None) == mm.MM_ERR_INVALID_ARG
    for name in ["mm_destroy_batch", "mm_batch_render"]:
        assert getattr(L, name)(None) == mm.MM_ERR_INVALID_ARG, name
    assert L.mm_batch_step_render(None, 0) == mm.MM_ERR_INVALID_ARG
    assert L.mm_batch_set_camera(None, 0, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_batch_read_frame(None, 0, None, 0) == mm.MM_ERR_INVALID_ARG
    assert L.mm_batch_set_tuning(None, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_batch_profile_begin(None, 4) == mm.MM_ERR_INVALID_ARG


def _c_layout(tmp_path, exprs):
    src = tmp_path / "layout2.c"
    fmt = " ".join(["%zu"] * len(exprs))
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "mm.h"\n'
                   'int main(void){printf("' + fmt + '\\n", ' + ", ".join(exprs) + ");return 0;}\n")
    exe = tmp_path / "layout2"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return [int(x) for x in out]


def test_batch_struct_layouts_match_the_header(tmp_path):
    structs = {
        "mm_tuning": mm.mm_tuning,
        "mm_cloud_desc": mm.mm_cloud_desc,
        "mm_batch_view_desc": mm.mm_batch_view_desc,
        "mm_batch_desc": mm.mm_batch_desc,
        "mm_batch_tuning": mm.mm_batch_tuning,
        "mm_colour_desc": mm.mm_colour_desc,
        "mm_grid_desc": mm.mm_grid_desc,
        "mm_edges_desc": mm.mm_edges_desc,
    }
    exprs, expect = [], []
    for cname, py in structs.items():
        for fname, _ in py._fields_:
            exprs.append(f"offsetof({cname}, {fname})")
            expect.append(getattr(py, fname).offset)
        exprs.append(f"sizeof({cname})")
        expect.append(C.sizeof(py))
    assert _c_layout(tmp_path, exprs) == expect


def test_server_calls_reject_null_arguments_without_a_device():
    L = mm.lib()
    assert L.mm_create_server(None, None, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_destroy_server(None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_server_add_cloud(None, None, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_server_submit(None, 0, 0, None, 2, 2, None, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_server_poll(None, 1, None, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_server_wait(None, 1, None) == mm.MM_ERR_INVALID_ARG
    assert L.mm_server_close_session(None, 0) == mm.MM_ERR_INVALID_ARG
    assert L.mm_server_stats_get(None, None) == mm.MM_ERR_INVALID_ARG


def test_server_struct_layouts_match_the_header(tmp_path):
    exprs, expect = [], []
    for cname, py in {"mm_server_desc": mm.mm_server_desc,
                      "mm_server_stats": mm.mm_server_stats}.items():
        for fname, _ in py._fields_:
            exprs.append(f"offsetof({cname}, {fname})")
            expect.append(getattr(py, fname).offset)
        exprs.append(f"sizeof({cname})")
        expect.append(C.sizeof(py))
    assert _c_layout(tmp_path, exprs) == expect


def test_build_rejects_kernels_with_scratch():
    """The build reads hipcc's resource-usage remarks and refuses a kernel that
    spills registers to scratch (the kernels are written to need none)."""
    from paper_2504_20937_amd import build
    remarks = "\n".join([
        "a.hip:1:1: remark: Function Name: good_kernel [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     VGPRs: 64 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark: Function Name: bad_kernel [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     VGPRs: 128 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     ScratchSize [bytes/lane]: 12 [-Rpass-analysis=kernel-resource-usage]",
    ])
    assert build._spilling_kernels(remarks) == ["bad_kernel (12 B/lane)"]
    assert build._spilling_kernels(remarks.split("\na.hip:9")[0]) == []
