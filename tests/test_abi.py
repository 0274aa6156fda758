"""The C-ABI library loads on the host and exports every function that
include/gic.h declares; the parameter struct's layout matches the binding;
host-side argument checks reject bad parameters before touching a device.
No compute calls: these run without a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2504_00745_amd import gic, workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gic.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:gic_status|int64_t|const char \*)\s+(gic_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_function():
    L = gic.lib()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    # and nothing is declared that the binding does not know about
    nm = subprocess.run(["nm", "-D", "--defined-only", gic.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\bT (gic_\w+)", nm.stdout))
    assert set(names) <= exported


def declared_arity():
    """Number of parameters of each function the header declares."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for m in re.finditer(r"^\s*(?:gic_status|int64_t|const char \*)\s+(gic_\w+)\s*\(([^;]*?)\)\s*;", src, flags=re.M | re.S):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_signatures_match_header():
    """The binding declares every function with as many arguments as the
    header does (a wrong count would pass garbage through ctypes)."""
    L = gic.lib()
    ar = declared_arity()
    assert len(ar) == len(declared_functions())
    for name, k in ar.items():
        f = getattr(L, name)
        assert f.argtypes is not None and len(f.argtypes) == k, (name, k, f.argtypes)


def test_params_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout.c"
    fields = [f[0] for f in gic.gic_params._fields_]
    body = "\n".join(f'printf("%zu\\n", offsetof(gic_params, {f}));' for f in fields)
    prog.write_text(f'#include <stdio.h>\n#include <stddef.h>\n#include "gic.h"\n'
                    f'int main(void){{printf("%zu\\n", sizeof(gic_params));\n{body}\nreturn 0;}}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(prog)], check=True)
    out = [int(t) for t in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert out[0] == C.sizeof(gic.gic_params)
    assert out[1:] == [getattr(gic.gic_params, f).offset for f in fields]


@pytest.mark.parametrize("name", wl.WORKLOADS)
def test_key_space_of_workloads(name):
    p = wl.spec(name)["params"]
    gp = gic.make_params(p, "fp32", p["cell"] / 2)
    K = gic.lib().gic_key_space(C.byref(gp))
    nb = [(a + 3) // 4 for a in p["nc"]]
    assert K == nb[0] * nb[1] * nb[2] * 64
    import oracle
    assert K == oracle.key_space(p)


def test_invalid_parameters_rejected_on_host():
    L = gic.lib()
    p = wl.spec("c1")["params"]
    h = C.c_void_p()
    bad = [dict(cell=0.001), dict(restitution=0.0), dict(restitution=1.5), dict(dt=0.0), dict(kn=-1.0),
           dict(nc=[64, 32, 32]), dict(walls=0x40)]
    for over in bad:
        q = dict(p)
        q.update(over)
        gp = gic.make_params(q, "fp64", 0.01)
        assert L.gic_key_space(C.byref(gp)) == -1, over
        assert L.gic_create(C.byref(gp), 10, C.byref(h)) == 1, over
    gp = gic.make_params(p, "fp64", 0.011)  # cell 0.02 < 2 r_max
    assert L.gic_create(C.byref(gp), 10, C.byref(h)) == 1
    gp = gic.make_params(p, "fp64", 0.01)
    gp.precision = 7
    assert L.gic_create(C.byref(gp), 10, C.byref(h)) == 1
    assert L.gic_create(C.byref(gic.make_params(p, "fp64", 0.01)), -1, C.byref(h)) == 1
    assert L.gic_destroy(None) == 1
