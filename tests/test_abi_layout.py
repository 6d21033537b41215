"""The ctypes mirrors of the ABI structs in paper_1202_6158_amd/di.py have the
size and field offsets that a C compiler gives the structs of include/di.h
(a small C program built with gcc prints them).  No GPU, no library call."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# ctypes class in di.py -> C struct in di.h (field names are the same)
PAIRS = [("Tune", "di_tune"), ("TuneTrial", "di_tune_trial"), ("Opts", "di_opts"),
         ("Stats", "di_stats"), ("ServerOpts", "di_server_opts"), ("Result", "di_result"),
         ("ServerMetrics", "di_server_metrics")]


def _binding_module():
    """di.py without loading libdi.so: its struct classes only."""
    import ctypes
    src = open(os.path.join(ROOT, "paper_1202_6158_amd", "di.py")).read()
    ns = {"ctypes": ctypes}
    for name, _ in PAIRS:
        start = src.index("class %s(ctypes.Structure):" % name)
        end = src.index("\n\n\n", start)
        exec(compile(src[start:end], "di.py:" + name, "exec"), ns)  # class bodies only
    return ns


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    ns = _binding_module()
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "di.h"', "int main(void) {"]
    for py, c in PAIRS:
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (c, c))
        for f in ns[py]._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (c, f[0], c, f[0]))
    lines.append("  return 0;\n}")
    d = tmp_path_factory.mktemp("abi")
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        c, field, v = line.split()
        table[(c, field)] = int(v)
    return ns, table


@pytest.mark.parametrize("py,c", PAIRS)
def test_struct_mirrors_match_the_header(c_layout, py, c):
    import ctypes
    ns, table = c_layout
    cls = ns[py]
    assert ctypes.sizeof(cls) == table[(c, "size")], (py, c)
    for f in cls._fields_:
        assert getattr(cls, f[0]).offset == table[(c, f[0])], (py, f[0])
