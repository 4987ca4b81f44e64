"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "osam.h")
LIB = os.path.join(ROOT, "paper_2511_20687_amd", "libosam.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary_calls():
    names = _declared()
    for n in ("create_subdomain", "learn_opinf", "schwarz_step", "run"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libosam.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libosam.so not built")
def test_binding_declares_the_same_symbols():
    from paper_2511_20687_amd import osam
    assert sorted(osam.EXPORTED) == _declared()
    lib = osam.load_library()
    assert lib.osam_version() >= 10000


# header struct -> ctypes class of the binding
_STRUCTS = {"osam_subdomain_desc": "SubdomainDesc", "osam_record": "Record", "osam_opinf_desc": "OpinfDesc",
            "osam_schwarz_opts": "SchwarzOpts", "osam_instance_info": "InstanceInfo", "osam_misfit": "Misfit",
            "osam_grads": "Grads", "osam_tuning": "Tuning"}


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every struct the binding marshals has the header's size and field offsets (a C program
    built against include/osam.h prints them; gcc, no GPU)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    from paper_2511_20687_amd import osam
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "osam.h"', 'int main(void) {']
    for cname, pyname in _STRUCTS.items():
        cls = getattr(osam, pyname)
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.rsplit(" ", 1)[0].split(" ")): int(l.rsplit(" ", 1)[1]) for l in out if l}
    for cname, pyname in _STRUCTS.items():
        cls = getattr(osam, pyname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert got[(cname, field)] == getattr(cls, field).offset, (cname, field)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libosam.so not built")
def test_binding_argument_counts_match_the_header():
    """Each declared call takes as many arguments in the binding as in the header."""
    from paper_2511_20687_amd import osam
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    protos = dict(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(([^)]*)\)\s*;", txt, flags=re.M))
    lib = osam.load_library()
    for name in osam.EXPORTED:
        params = protos[name].strip()
        n = 0 if params in ("", "void") else params.count(",") + 1
        argtypes = getattr(lib, name).argtypes
        assert len(argtypes or ()) == n, (name, n, argtypes)


def test_binding_rejects_bad_device_buffers():
    """The binding checks every device buffer it hands to the library (dtype of the context
    precision, contiguity, exact shape, device) before any pointer crosses the ABI: a wrong
    tensor would otherwise become out-of-bounds device reads or writes."""
    import torch
    from paper_2511_20687_amd.osam import Context
    ctx = object.__new__(Context)          # no device needed for the checks themselves
    ctx.precision, ctx.device, ctx.batch = "f32", 0, 2
    good = torch.zeros((2, 5, 7), dtype=torch.float32)
    with pytest.raises(ValueError, match="dtype"):
        ctx._check_buffer("u", good.double(), (2, 5, 7))
    with pytest.raises(ValueError, match="contiguous"):
        ctx._check_buffer("u", torch.zeros((2, 7, 5)).transpose(1, 2), (2, 5, 7))
    with pytest.raises(ValueError, match="shape"):
        ctx._check_buffer("u", good, (2, 5, 8))
    with pytest.raises(ValueError, match="shape"):
        ctx._check_buffer("u", good[0], (2, 5, 7))
    with pytest.raises(ValueError, match="cuda:0"):
        ctx._check_buffer("u", good, (2, 5, 7))
    with pytest.raises(ValueError, match="torch tensor"):
        ctx._check_buffer("u", good.numpy(), (2, 5, 7))
    ctx._check_buffer("u", None, (2, 5, 7))  # absent buffers are allowed
