"""The C-ABI library loads and exports every symbol include/qsim.h declares.

CPU only: no call here touches a GPU.
"""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import circuitgen as cg
import paper_quant_ph_9804039_amd as q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qsim.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qsim3?_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    if not os.path.exists(q.LIB_PATH):
        pytest.skip("libqsim.so not built (run __graft_entry__.build())")
    return q.LIB_PATH


def test_header_declares_the_contract():
    names = _declared()
    for must in ["qsim_create", "qsim_apply_circuit", "qsim_inject_errors", "qsim_fidelity",
                 "qsim_probs", "qsim_run_trials", "qsim_destroy", "qsim_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol(libpath):
    L = ctypes.CDLL(libpath)
    for name in _declared():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (qsim3?_\w+)", out))
    assert set(_declared()) <= exported
    assert set(q.EXPORTED) == set(_declared())


def test_binding_loads_and_reports_errors_as_text(libpath):
    L = q.lib()
    assert isinstance(L.qsim_last_error(), bytes)


def test_struct_layouts(tmp_path):
    assert cg.GATE_DTYPE.itemsize == 24
    text = open(HEADER).read()
    assert "double theta;" in text and "uint32_t kind;" in text
    # every struct the binding mirrors has the size the C compiler gives it
    names = ["qsim_gate", "qsim_error_model", "qsim_options", "qsim_stats", "qsim_pass_info",
             "qsim_request", "qsim_result", "qsim_serve_options", "qsim3_pulse"]
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include "qsim.h"\nint main(void) {\n' +
                   "".join(f'printf("%zu\\n", sizeof({n}));\n' for n in names) +
                   "return 0; }\n")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    sizes = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                            check=True).stdout.split()]
    mirror = {"qsim_gate": cg.GATE_DTYPE.itemsize}
    for n in names[1:]:
        mirror[n] = ctypes.sizeof(getattr(q, n))
    assert sizes == [mirror[n] for n in names]


def test_argument_errors_without_gpu(libpath):
    # rejected before any device call: no GPU needed
    h = ctypes.c_void_p()
    L = q.lib()
    assert L.qsim_create(0, 0, None, ctypes.byref(h)) == q.QSIM_EINVAL
    assert b"num_qubits" in L.qsim_last_error()
    assert L.qsim_create(35, 0, None, ctypes.byref(h)) == q.QSIM_EINVAL
    assert L.qsim_create(4, 7, None, ctypes.byref(h)) == q.QSIM_EINVAL
    assert L.qsim_create(4, 0, None, None) == q.QSIM_EINVAL
    g = np.zeros(1, dtype=cg.GATE_DTYPE)
    out = np.zeros(4)
    em = q.qsim_error_model(0.1, 0, 0, 1, 0)
    assert L.qsim_run_trials(g.ctypes.data, 1, 40, 0, ctypes.byref(em), 4,
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == q.QSIM_EINVAL
    assert L.qsim_destroy(None) == q.QSIM_OK


def test_host_memory_exhaustion_is_a_status_not_an_abort(libpath, tmp_path):
    """No C++ exception crosses the C-ABI: qsim_plan on a circuit whose
    lowered operation stream cannot fit the address space it is given (every
    qubit flips after every gate) returns QSIM_ENOMEM with a message instead
    of terminating the process.  Run in a child process under RLIMIT_AS."""
    script = tmp_path / "enomem.py"
    script.write_text(f'''
import ctypes, resource, sys
sys.path.insert(0, {ROOT!r})
import numpy as np
import circuitgen as cg
import paper_quant_ph_9804039_amd as q
L = q.lib()
gates = cg.random_circuit(30, 200000, 1)
em = q.qsim_error_model(0.0, 1.0, 1.0, 1, 0)
vm = [int(l.split()[1]) for l in open("/proc/self/status") if l.startswith("VmSize")][0] * 1024
soft, hard = resource.getrlimit(resource.RLIMIT_AS)
resource.setrlimit(resource.RLIMIT_AS, (vm + (512 << 20), hard))
npass, nops = ctypes.c_size_t(), ctypes.c_size_t()
rc = L.qsim_plan(30, 0, None, gates.ctypes.data, len(gates), ctypes.byref(em), 0, None, 0,
                 ctypes.byref(npass), ctypes.byref(nops), None, 0)
print(rc, L.qsim_last_error().decode())
''')
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    rc, msg = r.stdout.split(" ", 1)
    assert int(rc) == q.QSIM_ENOMEM, r.stdout
    assert "qsim_plan" in msg and "memory" in msg
