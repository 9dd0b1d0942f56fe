"""Host-side checks of the C ABI: the library loads without a GPU, exports
every function include/elbm.h declares, and validates arguments before any
device work."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1612_05404_amd import elbm
    if not os.path.exists(elbm.LIB_PATH):
        from paper_1612_05404_amd import build
        build.build()
    return elbm.load()


def _declared():
    src = open(os.path.join(ROOT, "include", "elbm.h")).read()
    # function declarations: a line that starts with a type and names elbm_*(
    decl = re.compile(r"^(?:const\s+)?[a-z_0-9]+\s*\*?\s*(elbm_[a-z_0-9]+)\s*\(", re.M)
    return sorted(set(decl.findall(src)))


def test_exports_every_declared_symbol(lib):
    from paper_1612_05404_amd import elbm
    names = _declared()
    assert len(names) >= 15
    assert sorted(elbm.SYMBOLS) == names
    for n in names:
        assert hasattr(lib, n), n


def test_abi_version(lib):
    from paper_1612_05404_amd import elbm
    assert lib.elbm_abi_version() == elbm.ABI_VERSION == 7


def test_struct_layouts_match_the_header(tmp_path):
    # the binding's structures have the sizes and field offsets the C compiler
    # gives the header's (a small C program built against include/elbm.h)
    import os
    import subprocess
    from paper_1612_05404_amd import elbm
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    structs = {"elbm_params": elbm.elbm_params, "elbm_box": elbm.elbm_box, "elbm_diag": elbm.elbm_diag,
               "elbm_launch": elbm.elbm_launch}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "elbm.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(root, "include"), "-o", str(exe), str(src)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(out[name]) == ct.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(out[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)


def _params(**kw):
    from paper_1612_05404_amd import elbm, inputs
    p = inputs.base_params(**kw)
    return elbm.make_params(p, elbm.STORAGE_F64), p


def _boxes(p, *shapes):
    from paper_1612_05404_amd import elbm, inputs
    bs = [inputs.droplet_box(*s, 3.0, seed=1) for s in shapes]
    return (elbm.elbm_box * len(bs))(*[elbm.make_box(p, b) for b in bs])


def test_create_and_layout_without_gpu(lib):
    P, p = _params()
    B = _boxes(p, (16, 16, 16), (10, 6, 8))
    h = ct.c_void_p()
    assert lib.elbm_create(ct.byref(P), B, 2, ct.byref(h)) == 0
    nb = ct.c_size_t()
    assert lib.elbm_required_bytes(h, ct.byref(nb)) == 0
    # two 19-direction double buffers of 2 components over 4096 + 512 padded nodes at least
    assert nb.value >= 2 * 2 * 19 * (4096 + 512) * 8
    # state calls before bind are refused
    assert lib.elbm_step(h, 1, 0) == -7
    assert lib.elbm_sync(h) == -7
    assert b"bound" in lib.elbm_last_error(h)
    lib.elbm_destroy(h)


@pytest.mark.parametrize("field,value", [("ncomp", 3), ("storage", 5), ("sor_sweeps", -1), ("newton_max", 0),
                                         ("charge_model", 7), ("alpha_guess", 9), ("strict", 4), ("strict", -1),
                                         ("alpha_iter", 2), ("sor_tol", -1e-3), ("sor_check_every", -2),
                                         ("inlet_mode", 4), ("inlet_mode", -1)])
def test_create_rejects_bad_params(lib, field, value):
    P, p = _params()
    setattr(P, field, value)
    B = _boxes(p, (8, 8, 8))
    h = ct.c_void_p()
    assert lib.elbm_create(ct.byref(P), B, 1, ct.byref(h)) == -1
    assert not h.value


def test_create_rejects_bad_boxes(lib):
    P, p = _params()
    h = ct.c_void_p()
    B = _boxes(p, (7, 8, 8))          # odd periodic length breaks the red-black colouring
    assert lib.elbm_create(ct.byref(P), B, 1, ct.byref(h)) == -1
    B = _boxes(p, (8, 8, 8))
    B[0].sor_omega = 2.0
    assert lib.elbm_create(ct.byref(P), B, 1, ct.byref(h)) == -1
    assert lib.elbm_create(ct.byref(P), B, 0, ct.byref(h)) == -1
    assert lib.elbm_create(None, B, 1, ct.byref(h)) == -1


def test_create_checks_the_inlet_mode_against_the_lattice(lib):
    # the adaptive inlet measures along x, y or z; a D2Q9 box has no z axis
    from paper_1612_05404_amd import elbm, inputs
    wl = inputs.paper_jet_2d(n=32, diameter=8, nozzle_len=6, wall=2)
    B = (elbm.elbm_box * 1)(elbm.make_box(wl.params, wl.boxes[0]))
    h = ct.c_void_p()
    for mode, ok in ((elbm.INLET_ADAPTIVE_X, True), (elbm.INLET_ADAPTIVE_Y, True), (elbm.INLET_ADAPTIVE_Z, False),
                     (elbm.INLET_NEIGHBOUR, True)):
        P = elbm.make_params(wl.params.with_(inlet_mode=mode), elbm.STORAGE_F64)
        st = lib.elbm_create(ct.byref(P), B, 1, ct.byref(h))
        assert (st == 0) == ok, mode
        if st == 0:
            lib.elbm_destroy(h)
            h = ct.c_void_p()
