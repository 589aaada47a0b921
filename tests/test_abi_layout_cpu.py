"""The ctypes structures of the binding against the C header: every field
the header declares, by name and in order, and a small C program built with
gcc from include/ri.h that prints the size of every ABI struct and the offset
and size of every field, which must equal what ctypes computes for the
binding's declarations.  A field added on one side only, or a changed type,
fails here before any call could read or write past it."""

import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_2412_14975_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = ("ri_build_opts", "ri_result", "ri_tuning", "ri_info_t", "ri_request", "ri_batch_info",
           "ri_batch_opts", "ri_batch_group", "ri_batch_tuning")


def _header_fields():
    """Field names of every `typedef struct { ... } name;` in the header, in
    order (comments removed; one declarator per line)."""
    text = open(os.path.join(ROOT, "include", "ri.h")).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(\w+)\s*;", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if decl:
                fields.append(re.match(r".*?(\w+)\s*(\[[^\]]*\])?$", decl, flags=re.S).group(1))
        out[name] = fields
    return out


def test_binding_declares_every_header_field():
    hdr = _header_fields()
    assert set(STRUCTS) <= set(hdr), set(STRUCTS) - set(hdr)
    for name in STRUCTS:
        assert [f for f, _ in getattr(B, name)._fields_] == hdr[name], name


def _c_source():
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ri.h"', "int main(void) {"]
    for name in STRUCTS:
        cls = getattr(B, name)
        lines.append(f'    printf("{name} %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("{name}.{field} %zu %zu\\n", offsetof({name}, {field}), '
                         f'sizeof((({name} *)0)->{field}));')
    lines += ["    return 0;", "}"]
    return "\n".join(lines) + "\n"


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_binding_structs_match_the_header(tmp_path):
    src = tmp_path / "layout.c"
    exe = tmp_path / "layout"
    src.write_text(_c_source())
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        key, *vals = line.split()
        got[key] = tuple(int(v) for v in vals)
    for name in STRUCTS:
        cls = getattr(B, name)
        assert got[name] == (ctypes.sizeof(cls),), name
        for field, ctype in cls._fields_:
            desc = getattr(cls, field)
            assert got[f"{name}.{field}"] == (desc.offset, desc.size), (name, field)
