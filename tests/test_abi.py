"""The C-ABI library builds, loads on the host and exports every function that
include/stba.h declares (no compute calls: there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stba.h")
LIB = os.path.join(ROOT, "paper_2008_00446_amd", "libstba.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int|size_t|char)\s*\*?\s*(stba_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for fn in ("stba_residual_jacobian", "stba_build_cluster_rcs", "stba_solve_clusters", "stba_lm_step"):
        assert fn in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libstba.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.stba_version.restype = ctypes.c_char_p
    assert lib.stba_version().startswith(b"stba")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libstba.so not built")
def test_binding_names_match_header_and_host_checks():
    import paper_2008_00446_amd as P
    from paper_2008_00446_amd import binding as B
    B.load_library()
    for n in declared_functions():
        assert hasattr(B, n), n
    # host-side argument checks return before touching the device
    lib = B.load_library()
    assert lib.stba_workspace_bytes(None, None, 0) == 0
    assert lib.stba_lm_init(None, 1e-4, 0.1, None) == -1
    assert P.stba_phase_name(0) == "clusters" and P.stba_phase_name(99) == ""


def test_ctypes_structs_match_the_c_layout(tmp_path):
    """Every struct the binding mirrors has the header's size and field offsets
    (the header compiled by the host C compiler)."""
    import shutil
    import subprocess

    from paper_2008_00446_amd import binding as B

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    structs = {"stba_problem": B.StbaProblem, "stba_dims": B.StbaDims, "stba_sample": B.StbaSample,
               "stba_damping": B.StbaDamping, "stba_lm_state": B.StbaLmState, "stba_rcs": B.StbaRcs}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "stba.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            cf = "lambda" if fname == "lambda_" else fname
            lines.append(f'    printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        cname, what, val = line.split()
        py = structs[cname]
        got = ctypes.sizeof(py) if what == "size" else getattr(py, what).offset
        assert got == int(val), (cname, what, got, val)


def test_product_path_never_imports_the_oracle_and_has_no_fallback(tmp_path):
    """Importing and using the package's host side loads no oracle module, and a
    missing library is an error, not a switch to some other path."""
    import subprocess
    import sys

    code = (
        "import sys\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import paper_2008_00446_amd as P\n"
        "from paper_2008_00446_amd import binding as B, solver\n"
        "assert not any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules), 'oracle imported'\n"
        "try:\n"
        f"    B._lib = None\n"
        f"    B.load_library({str(tmp_path / 'missing.so')!r})\n"
        "except ImportError:\n"
        "    print('raised')\n"
    )
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "raised"
    # and the package's sources do not name the oracle at all
    pkg = os.path.join(ROOT, "paper_2008_00446_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_launch_settings_are_checked_on_the_host():
    """stba_workspace_bytes (host, pure) returns 0 for dims whose factorisation
    form or Schur workgroup count is out of range."""
    import ctypes
    import paper_2008_00446_amd as S
    from paper_2008_00446_amd import binding as B
    lib = S.load_library()
    prob = B.StbaProblem(10, 10, 40, ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256),
                         ctypes.c_void_p(256), ctypes.c_void_p(256), 0.0)
    ok = B.StbaDims(100, 4, 5, 0, 0)
    assert lib.stba_workspace_bytes(ctypes.byref(prob), ctypes.byref(ok), 0) > 0
    for form, blocks in [(4, 0), (-1, 0), (0, 7), (0, 65537)]:
        bad = B.StbaDims(100, 4, 5, form, blocks)
        assert lib.stba_workspace_bytes(ctypes.byref(prob), ctypes.byref(bad), 0) == 0
    assert lib.stba_workspace_bytes(ctypes.byref(prob), ctypes.byref(B.StbaDims(100, 4, 5, 3, 8)), 0) > 0
