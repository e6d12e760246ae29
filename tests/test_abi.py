"""The C-ABI library: it loads, exports every symbol include/acse.h declares,
and rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2604_02550_amd", "libacse.so")
HEADER = os.path.join(ROOT, "include", "acse.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(acse_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libacse.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "acse_residual" in names and "acse_step" in names and "acse_energy" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_every_export():
    import importlib.util
    spec = importlib.util.find_spec("paper_2604_02550_amd")
    src = open(spec.origin).read()
    for n in _declared():
        assert f'"{n}"' in src, n


def test_status_strings(lib):
    lib.acse_status_str.restype = ctypes.c_char_p
    assert lib.acse_status_str(0) == b"ACSE_OK"
    assert lib.acse_status_str(4) == b"ACSE_ERR_UNSUPPORTED"
    assert lib.acse_status_str(7) == b"ACSE_ERR_NONFINITE"
    assert lib.acse_status_str(99) == b"ACSE_ERR_UNKNOWN"


def test_argument_errors_without_device(lib):
    P = ctypes.c_void_p
    lib.acse_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P, ctypes.c_int32]
    h = P()
    assert lib.acse_create(None, 0, None, 10) == 1            # ACSE_ERR_ARG
    assert lib.acse_create(ctypes.byref(h), 0, None, 1) == 2  # r_max < 2
    assert lib.acse_create(ctypes.byref(h), 0, None, 10 ** 4) == 2
    lib.acse_destroy.argtypes = [P]
    assert lib.acse_destroy(None) == 1
    lib.acse_residual.argtypes = [P] * 5 + [ctypes.POINTER(ctypes.c_double)]
    assert lib.acse_residual(None, None, None, None, None, None) == 1
    lib.acse_energy.argtypes = [P, P, ctypes.POINTER(ctypes.c_double)]
    assert lib.acse_energy(None, None, None) == 1
    lib.acse_last_error.restype = ctypes.c_char_p
    lib.acse_last_error.argtypes = [P]
    # with no context: the detail of the last failing context-free call on this
    # thread (none has failed here yet, or acse_residual_noalloc's if one has)
    assert isinstance(lib.acse_last_error(None), bytes)


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes structs have the C header's sizes and field offsets
    (checked with a small C program built by gcc against include/acse.h)."""
    import shutil
    import subprocess
    import paper_2604_02550_amd as acse
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = tmp_path / "layout.c"
    structs = (("acse_problem", acse.Problem), ("acse_problem_spin", acse.ProblemSpin), ("acse_options", acse.Options),
               ("acse_profile_data", acse.ProfileData), ("acse_solve_options", acse.SolveOptions),
               ("acse_trial", acse.Trial), ("acse_solve_result", acse.SolveResult))
    fields = {st: [f for f, _ in cls._fields_] for st, cls in structs}
    lines = ["#include <stdio.h>", "#include <stddef.h>", "#include \"acse.h\"", "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'  printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'  printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                               text=True).stdout.split("\n") if line)
    for st, cls in structs:
        assert int(out[st]) == ctypes.sizeof(cls), st
        for f, _ in cls._fields_:
            assert int(out[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)


def test_trajectory_from_trials():
    """lambda = sum of the accepted step sizes; E and log10 ||R|| of the input
    state and of each accepted trial (rejected trials are skipped)."""
    import math
    import paper_2604_02550_amd as acse
    res = dict(energy0=-1.0, norm2_0=100.0,
               trials=[(0.1, -2.0, 50.0, 0, False), (0.05, -1.5, 81.0, 0, True),
                       (0.05, -1.8, 64.0, 1, True)])
    t = acse.trajectory(res)
    assert t == [(0.0, -1.0, 1.0), (0.05, -1.5, math.log10(9.0)), (0.1, -1.8, math.log10(8.0))]


def test_noalloc_argument_errors_without_device(lib):
    """acse_residual_noalloc rejects a missing problem and sizes beyond its
    maximum before it touches a device; acse_last_error(NULL) names the cause."""
    P = ctypes.c_void_p
    lib.acse_residual_noalloc.argtypes = [P] * 6
    lib.acse_last_error.argtypes = [P]
    lib.acse_last_error.restype = ctypes.c_char_p
    assert lib.acse_residual_noalloc(None, None, None, None, None, None) == 1   # ACSE_ERR_ARG
    assert b"problem is NULL" in lib.acse_last_error(None)

    class Problem(ctypes.Structure):
        _fields_ = [("r", ctypes.c_int32), ("n_alpha", ctypes.c_int32), ("n_beta", ctypes.c_int32),
                    ("h", P), ("V", P), ("d1", P), ("d2aa", P), ("d2ab", P)]

    for r in (1, 17, 50):
        prob = Problem(r, 2, 2, None, None, None, None, None)
        assert lib.acse_residual_noalloc(None, ctypes.byref(prob), None, None, None, None) == 2
        assert b"outside [2, 16]" in lib.acse_last_error(None)
