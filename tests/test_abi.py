"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every declared
function, validates its arguments and computes the host-only quantities."""
import ctypes as C
import math
import os
import re

import pytest

from paper_2607_17929_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_function_is_exported():
    lib = L.load()
    names = _declared()
    assert set(names) == set(L.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_query_workspace_and_validation():
    lib = L.load()
    cfg = L.PMConfig(n_mesh=64, precision=L.PM_FP32, n_particles=64 ** 3, box_mpch=256.0, physics=L.PM_FULL, flags=0)
    b = C.c_size_t()
    assert lib.pm_query_workspace(C.byref(cfg), C.byref(b)) == L.PM_OK
    n3 = 64 ** 3
    # at least: two particle buffers (40 B each), 10 deposits, 7 real fields, 10 + 4 half spectra
    assert b.value > n3 * (2 * 40 + 4 * 17) + 14 * 64 * 64 * 33 * 8
    bad = L.PMConfig(n_mesh=48, precision=L.PM_FP32, n_particles=10, box_mpch=256.0, physics=L.PM_FULL, flags=0)
    assert lib.pm_query_workspace(C.byref(bad), C.byref(b)) == L.PM_ERANGE
    bad.n_mesh = 2048
    assert lib.pm_query_workspace(C.byref(bad), C.byref(b)) == L.PM_ERANGE
    bad.n_mesh, bad.precision = 64, 7
    assert lib.pm_query_workspace(C.byref(bad), C.byref(b)) == L.PM_EINVAL
    ctx = C.c_void_p()
    assert lib.pm_create(C.byref(cfg), None, 0, None, C.byref(ctx)) == L.PM_EWORKSPACE
    assert lib.pm_create(C.byref(cfg), C.c_void_p(256), 16, None, C.byref(ctx)) == L.PM_EWORKSPACE
    assert lib.pm_deposit(None) == L.PM_EINVAL
    assert lib.pm_status_string(L.PM_ESTATE) == b"call out of order"


def test_background_host_functions():
    lib = L.load()
    cfg = L.PMConfig(n_mesh=32, precision=L.PM_FP64, n_particles=1, box_mpch=320.0, physics=L.PM_SCALAR, flags=0)
    tau = C.c_double()
    assert lib.pm_tau_of_a(C.byref(cfg), 0.02, C.byref(tau)) == L.PM_OK
    a, h = C.c_double(), C.c_double()
    assert lib.pm_background(C.byref(cfg), tau.value, C.byref(a), C.byref(h)) == L.PM_OK
    assert abs(a.value - 0.02) < 1e-15
    # Einstein-de Sitter: H_conf = H0 / sqrt(a), H0 = box / (c / 100 km/s/Mpc)
    assert abs(h.value - (320.0 / 2997.92458) / math.sqrt(0.02)) < 1e-12
    assert lib.pm_background(C.byref(cfg), -1.0, C.byref(a), C.byref(h)) == L.PM_EINVAL


def _header_constants():
    src = open(os.path.join(ROOT, "include", "pm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return {k: int(v) for k, v in re.findall(r"\b(PM_[A-Z0-9_]+)\s*=\s*(-?\d+)u?\b", src)}


def test_copy_probe_rejects_bad_arguments():
    """pm_copy_probe validates its arguments on the host before any device call: sizes that are zero or not a
    multiple of 16, pointers not aligned to 16 bytes, null pointers and reps < 1 give PM_EINVAL."""
    lib = L.load()
    ms = C.c_double()
    a, b = C.c_void_p(1 << 20), C.c_void_p(2 << 20)  # never dereferenced: every call below is rejected first
    assert lib.pm_copy_probe(a, b, 24, 1, None, C.byref(ms)) == L.PM_EINVAL
    assert lib.pm_copy_probe(a, b, 0, 1, None, C.byref(ms)) == L.PM_EINVAL
    assert lib.pm_copy_probe(C.c_void_p((1 << 20) + 8), b, 64, 1, None, C.byref(ms)) == L.PM_EINVAL
    assert lib.pm_copy_probe(a, C.c_void_p((2 << 20) + 4), 64, 1, None, C.byref(ms)) == L.PM_EINVAL
    assert lib.pm_copy_probe(None, b, 64, 1, None, C.byref(ms)) == L.PM_EINVAL
    assert lib.pm_copy_probe(a, b, 64, 0, None, C.byref(ms)) == L.PM_EINVAL
    assert lib.pm_copy_probe(a, b, 64, 1, None, None) == L.PM_EINVAL


def test_header_constants_match_the_binding():
    h = _header_constants()
    for name in ("PM_OK", "PM_EINVAL", "PM_EWORKSPACE", "PM_EHIP", "PM_ENAN", "PM_ESTATE", "PM_ERANGE",
                 "PM_EUNSUPPORTED", "PM_FP32", "PM_FP64", "PM_NEWTONIAN", "PM_SCALAR", "PM_FULL",
                 "PM_FLAG_TIMINGS", "PM_FLAG_CLOSURE", "PM_FLAG_B_PARABOLIC", "PM_FLAG_DETERMINISTIC", "PM_CLOSURE_NPARAM"):
        assert h[name] == getattr(L, name), name
    for name, fid in L.FIELDS.items():
        assert h["PM_FIELD_" + name.upper()] == fid, name
    assert h["PM_FIELD_COUNT"] == len(L.FIELDS)
    for i, name in enumerate(L.STAGES):
        assert h["PM_STAGE_" + name.upper()] == i, name
    assert h["PM_NSTAGES"] == len(L.STAGES)


def test_config_struct_layout_matches_c(tmp_path):
    """The ctypes pm_config has the C struct's size and field offsets (compiled with the host compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    fields = [f[0] for f in L.PMConfig._fields_]
    prog = tmp_path / "layout.c"
    prog.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"pm.h\"\nint main(void) {\n"
                    "  printf(\"%zu\\n\", sizeof(pm_config));\n"
                    + "".join(f"  printf(\"%zu\\n\", offsetof(pm_config, {f}));\n" for f in fields)
                    + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    out = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert out[0] == C.sizeof(L.PMConfig)
    for f, off in zip(fields, out[1:]):
        assert getattr(L.PMConfig, f).offset == off, f


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library there is no fallback: loading it raises, and so does creating a
    context (before any device work)."""
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "libgpm.so"))
    with pytest.raises(ImportError):
        L.load()
    from paper_2607_17929_amd import PMContext
    with pytest.raises(ImportError):
        PMContext(16, 8, 100.0, physics="scalar", precision="fp64")
