"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point include/gspm.h declares, reports a missing device cleanly,
and its host-only demagnetisation factors meet the closed forms."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2510_09812_amd import gspm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "gspm.h")).read()
    return sorted(set(re.findall(r"\b(gspm_[a-z_]+)\s*\(", text)) - {"gspm_ctx"})


def test_header_and_binding_agree():
    assert sorted(gspm.EXPORTS) == _declared()


def test_header_enum_values_match_the_binding():
    """Every GSPM_* enumerator and #define of the header has the value the
    binding's constant of the same name carries."""
    text = open(os.path.join(ROOT, "include", "gspm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)      # comments may hold braces
    values = {}
    for body in re.findall(r"typedef enum\s*\{(.*?)\}", text, re.S):
        nxt = 0
        for item in body.split(","):
            item = item.strip()
            if not item:
                continue
            m = re.match(r"(GSPM_\w+)\s*(?:=\s*(-?\d+))?$", item)
            assert m, item
            nxt = int(m.group(2)) if m.group(2) is not None else nxt
            values[m.group(1)] = nxt
            nxt += 1
    for name, val in re.findall(r"#define\s+(GSPM_\w+)\s+(\d+)\b", text):
        values[name] = int(val)
    checked = 0
    for name, val in values.items():
        if hasattr(gspm, name):
            assert getattr(gspm, name) == val, name
            checked += 1
    for name in ("GSPM_GS_START_LUMPED", "GSPM_GS_START_CORRECTED", "GSPM_MIXED", "GSPM_PRECOND_JACOBI",
                 "GSPM_REORDER_RCM", "GSPM_WARM_EXTRAPOLATE", "GSPM_MPNN_PARAMS"):
        assert name in values and hasattr(gspm, name), name
    assert checked >= 20


def test_struct_layouts_match_the_binding(tmp_path):
    """The ctypes structures of the binding have the size and field offsets
    the C compiler gives the header's structs (tests/host/abi_layout.c)."""
    import ctypes
    import shutil
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "abi_layout")
    subprocess.check_call([gcc, "-std=c11", "-I" + os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "host", "abi_layout.c"), "-o", exe])
    lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    seen = 0
    for line in filter(None, lines):
        struct, field, value = line.split()
        cls = getattr(gspm, struct)
        got = ctypes.sizeof(cls) if field == "sizeof" else getattr(cls, field).offset
        assert got == int(value), (struct, field, got, value)
        seen += 1
    # every ctypes field is covered by the C listing
    for cls in (gspm.gspm_create_opts, gspm.gspm_params, gspm.gspm_step_stats):
        names = {line.split()[1] for line in filter(None, lines) if line.split()[0] == cls.__name__}
        assert {f[0] for f in cls._fields_} <= names, cls.__name__
    assert seen >= 50


def test_library_exports_every_declared_symbol():
    lib = gspm.load()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", gspm.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (gspm_\w+)", out))
    assert set(_declared()) <= exported


def test_no_device_or_bad_options_fail_cleanly():
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    with pytest.raises(gspm.GspmError) as e:
        gspm.gspm_create(precision=7)
    assert e.value.status == gspm.GSPM_E_ARG
    with pytest.raises(gspm.GspmError) as e:
        gspm.gspm_create(block_nodes=100)
    assert e.value.status == gspm.GSPM_E_ARG
    if not has_gpu:
        with pytest.raises(gspm.GspmError) as e:
            gspm.gspm_create()
        assert e.value.status == gspm.GSPM_E_DEVICE
        assert "device" in gspm.gspm_last_error(None)


def test_demag_factors_closed_forms():
    assert np.allclose(gspm.gspm_demag_factors(2.0, 2.0, 2.0), 1.0 / 3.0, atol=1e-14)
    for mm in (1.5, 3.0, 10.0):
        Na = (mm / np.sqrt(mm * mm - 1) * np.log(mm + np.sqrt(mm * mm - 1)) - 1.0) / (mm * mm - 1)
        N = gspm.gspm_demag_factors(mm, 1.0, 1.0)
        assert abs(N[0] - Na) < 1e-13 and abs(N[1] - (1 - Na) / 2) < 1e-13
        Nc = mm * mm / (mm * mm - 1) * (1.0 - np.arcsin(np.sqrt(mm * mm - 1) / mm) / np.sqrt(mm * mm - 1))
        N = gspm.gspm_demag_factors(mm, mm, 1.0)
        assert abs(N[2] - Nc) < 1e-13
    N = gspm.gspm_demag_factors(3.0, 1.3, 0.6)
    assert abs(N.sum() - 1.0) < 1e-13
    with pytest.raises(gspm.GspmError):
        gspm.gspm_demag_factors(-1.0, 1.0, 1.0)


def test_create_option_checks_without_a_device():
    with pytest.raises(gspm.GspmError) as e:
        gspm.gspm_create(reorder=9)
    assert e.value.status == gspm.GSPM_E_ARG
    only_alloc = (gspm.DEV_ALLOC_FN(lambda n, u: None), None)
    opts = gspm.gspm_create_opts(0, 0, 0, 0, None, 0)
    opts.dev_alloc = only_alloc[0]
    import ctypes
    h = ctypes.c_void_p()
    assert gspm.load().gspm_create(ctypes.byref(h), ctypes.byref(opts)) == gspm.GSPM_E_ARG
