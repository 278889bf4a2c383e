"""The C-ABI library loads and exports every function include/fcd.h declares; host-side
argument checks reject bad input without touching a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2410_11129_amd import fcd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fcd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fcd_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(fcd.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = fcd.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the ctypes structs equal those a C compiler gives the
    header's structs."""
    structs = {"fcd_lattice": fcd.fcd_lattice, "fcd_params": fcd.fcd_params, "fcd_buffers": fcd.fcd_buffers}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fcd.h"', "int main(void) {"]
    for sname, cls in structs.items():
        lines.append(f'printf("{sname} size %zu\\n", sizeof({sname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{sname} {fname} %zu\\n", offsetof({sname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for sname, cls in structs.items():
        assert got[(sname, "size")] == C.sizeof(cls), sname
        for fname, _ in cls._fields_:
            assert got[(sname, fname)] == getattr(cls, fname).offset, (sname, fname)


def test_scratch_bytes_is_host_only():
    lat = fcd.fcd_lattice(200, 50, fcd.FCD_FP64, 256)
    assert fcd.fcd_scratch_bytes(lat) >= 50 * 8 * 8


def good_params():
    from fcd_inputs import single_channel_small
    from paper_2410_11129_amd.sim import make_params
    return make_params(single_channel_small())


@pytest.mark.parametrize("nx,ny,prec,pitch", [(201, 50, 0, 256), (2, 50, 0, 256), (200, 1, 0, 256),
                                              (200, 50, 0, 100), (200, 50, 7, 256)])
def test_bad_lattice_rejected_before_any_device_work(nx, ny, prec, pitch):
    lat = fcd.fcd_lattice(nx, ny, prec, pitch)
    buf = fcd.fcd_buffers()
    buf.dist[0], buf.dist[1], buf.phi, buf.psi, buf.scratch = 256, 512, 768, 1024, 1280
    h = C.c_void_p()
    st = fcd.lib().fcd_create(C.byref(lat), C.byref(good_params()), C.byref(buf), None, C.byref(h))
    assert st == fcd.FCD_ERR_ARG
    assert fcd.fcd_last_error()


def test_bad_params_and_null_buffers_rejected():
    lat = fcd.fcd_lattice(200, 50, fcd.FCD_FP64, 256)
    buf = fcd.fcd_buffers()
    h = C.c_void_p()
    st = fcd.lib().fcd_create(C.byref(lat), C.byref(good_params()), C.byref(buf), None, C.byref(h))
    assert st == fcd.FCD_ERR_ARG and "null" in fcd.fcd_last_error()
    p = good_params()
    p.sigma12, p.sigma13, p.sigma23 = 0.01, 0.02, 0.01  # gamma_2 = 0
    buf.dist[0], buf.dist[1], buf.phi, buf.psi, buf.scratch = 256, 512, 768, 1024, 1280
    st = fcd.lib().fcd_create(C.byref(lat), C.byref(p), C.byref(buf), None, C.byref(h))
    assert st == fcd.FCD_ERR_ARG and "gamma" in fcd.fcd_last_error()
    assert fcd.lib().fcd_step(None, 1) == fcd.FCD_ERR_ARG


def test_batch_schedule_calls_and_warm_start_order_validated_on_host():
    """Null batches and out-of-range settings are rejected before any device work."""
    L = fcd.lib()
    choice = (C.c_int32 * 5)()
    scales = (C.c_double * 2)(1.0, 0.9)
    out = (C.c_double * 4)()
    assert L.fcd_batch_set_schedule(None, 4, 8, 2) == fcd.FCD_ERR_ARG
    assert L.fcd_batch_set_tail_fusion(None, 4, 64) == fcd.FCD_ERR_ARG
    assert L.fcd_batch_autotune(None, 1, choice) == fcd.FCD_ERR_ARG
    assert L.fcd_batch_tune_omega(None, 4, 2, scales, out) == fcd.FCD_ERR_ARG
    lat = fcd.fcd_lattice(200, 50, fcd.FCD_FP64, 256)
    buf = fcd.fcd_buffers()
    buf.dist[0], buf.dist[1], buf.phi, buf.psi, buf.scratch = 256, 512, 768, 1024, 1280
    p = good_params()
    p.pot_coarse_sweeps = 0  # positive: times ny_c / 2; negative: an absolute count
    st = L.fcd_create(C.byref(lat), C.byref(p), C.byref(buf), None, C.byref(h := C.c_void_p()))
    assert st == fcd.FCD_ERR_ARG and "pot_coarse_sweeps" in fcd.fcd_last_error()
    p = good_params()
    p.pot_extrapolate = 4  # 0..3: none, linear, quadratic, cubic
    h = C.c_void_p()
    st = L.fcd_create(C.byref(lat), C.byref(p), C.byref(buf), None, C.byref(h))
    assert st == fcd.FCD_ERR_ARG and "pot_extrapolate" in fcd.fcd_last_error()


def test_divergence_guard_settings_validated_on_host():
    """The divergence guard's limit and check interval are checked before any device work;
    0 selects the defaults."""
    L = fcd.lib()
    lat = fcd.fcd_lattice(200, 50, fcd.FCD_FP64, 256)
    buf = fcd.fcd_buffers()
    buf.dist[0], buf.dist[1], buf.phi, buf.psi, buf.scratch = 256, 512, 768, 1024, 1280
    h = C.c_void_p()
    p = good_params()
    assert p.u_limit == 0.0 and p.div_check_every == 0
    p.u_limit = -0.1
    assert L.fcd_create(C.byref(lat), C.byref(p), C.byref(buf), None, C.byref(h)) == fcd.FCD_ERR_ARG
    assert "u_limit" in fcd.fcd_last_error()
    p = good_params()
    p.u_limit = float("nan")
    assert L.fcd_create(C.byref(lat), C.byref(p), C.byref(buf), None, C.byref(h)) == fcd.FCD_ERR_ARG
    p = good_params()
    p.div_check_every = -1
    assert L.fcd_create(C.byref(lat), C.byref(p), C.byref(buf), None, C.byref(h)) == fcd.FCD_ERR_ARG
    assert "div_check_every" in fcd.fcd_last_error()
    assert L.fcd_sync(None) == fcd.FCD_ERR_ARG


def test_noalloc_limit_matches_header_and_is_checked_on_host():
    """fcd_deformation_noalloc's row limit is the header's, and a larger lattice is rejected
    before any device work."""
    text = open(os.path.join(ROOT, "include", "fcd.h")).read()
    m = re.search(r"#define FCD_NOALLOC_MAX_NY (\d+)", text)
    assert m and int(m.group(1)) == fcd.FCD_NOALLOC_MAX_NY
    lat = fcd.fcd_lattice(8, fcd.FCD_NOALLOC_MAX_NY + 2, fcd.FCD_FP64, 8)
    st = fcd.lib().fcd_deformation_noalloc(C.byref(lat), C.c_void_p(256), None, C.c_void_p(512))
    assert st == fcd.FCD_ERR_ARG and "FCD_NOALLOC_MAX_NY" in fcd.fcd_last_error()
    assert fcd.lib().fcd_deformation_noalloc(C.byref(lat), None, None, None) == fcd.FCD_ERR_ARG
