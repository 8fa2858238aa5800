"""The C-ABI library loads, exports every symbol include/mcdc.h declares,
and rejects invalid descriptors before touching a device (CPU-only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcdc.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(mcdc_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ["mcdc_problem_create", "mcdc_problem_destroy", "mcdc_problem_tally_shape",
              "mcdc_run", "mcdc_set_weight_windows", "mcdc_last_error"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2305_07636_amd import _binding

    L = _binding.lib()
    for s in declared_symbols():
        assert hasattr(L, s), s
    assert set(_binding.EXPORTS) <= set(declared_symbols())


def _create(prob):
    from paper_2305_07636_amd import _binding as b

    d, keep = b.make_desc(prob)
    h = C.c_void_p()
    rc = b.lib().mcdc_problem_create(C.byref(d), C.byref(h))
    return rc, b.lib().mcdc_last_error().decode()


def _mutated(**changes):
    p = w.cfg3_lattice()
    for k, v in changes.items():
        if "." in k:
            a, b = k.split(".")
            p[a][b] = v
        else:
            p[k] = v
    return p


@pytest.mark.parametrize("change,needle", [
    ({"sigma_t": -np.ones((2, 7))}, "sigma_t"),
    ({"speed": np.zeros(7)}, "speed"),
    ({"material": np.full((1, 17, 17), 5, dtype=np.int32)}, "material"),
    ({"bc": np.array([0, 0, 0, 0, 0, 2], dtype=np.int32)}, "boundary"),
])
def test_invalid_descriptors_rejected(change, needle):
    rc, msg = _create(_mutated(**change))
    assert rc == -1 and needle in msg, (rc, msg)


def test_invalid_scattering_exceeds_total():
    p = w.cfg3_lattice()
    p["sigma_s"] = p["sigma_s"] * 10
    rc, msg = _create(p)
    assert rc == -1 and "scattering" in msg


def test_invalid_planes_and_time_edges():
    p = w.cfg3_lattice()
    p["planes"][0] = p["planes"][0][::-1].copy()
    assert _create(p)[0] == -1
    p = w.cfg2_slab_pulse()
    p["tally"]["time_edges"] = np.array([0.0, 1.0, 1.0])
    assert _create(p)[0] == -1
    p = w.cfg2_slab_pulse()
    p["source"]["group_pmf"] = np.array([0.5])
    rc, msg = _create(p)
    assert rc == -1 and "pmf" in msg
    p = w.cfg2_slab_pulse()
    p["source"]["lo"] = np.array([50.0, 0, 0])
    p["source"]["hi"] = np.array([50.0, 0, 0])
    rc, msg = _create(p)
    assert rc == -1 and "source" in msg
    p = w.cfg2_slab_pulse()
    p["tally"]["mesh"][0] = np.array([-1.0, 50.0])
    assert _create(p)[0] == -1


def test_run_rejects_bad_arguments():
    from paper_2305_07636_amd import _binding as b

    res = b.mcdc_result()
    assert b.lib().mcdc_run(None, 10, 1, None, C.byref(res)) == -1
    assert b.lib().mcdc_problem_destroy(None) == 0


def _fis(sf, nu, chi):
    return {"sigma_f": np.array([[sf]]), "nu": np.array([[nu]]), "chi": np.array([[chi]])}


@pytest.mark.parametrize("fission,needle", [
    (_fis(0.6, 2.0, 1.0), "exceeds"),          # sigma_s 0.5 + sigma_f 0.6 > sigma_t 1
    (_fis(0.1, 65.0, 1.0), "nu"),
    (_fis(-0.1, 2.0, 1.0), "sigma_f"),
    (_fis(0.1, 2.0, 0.9), "chi"),
])
def test_invalid_fission_rejected(fission, needle):
    p = w.reflective_box([1.0], [[0.5]], [1.0], fission=fission)
    rc, msg = _create(p)
    assert rc == -1 and needle in msg, (rc, msg)


@pytest.mark.parametrize("ic,needle", [
    ({"w_min": 0.0, "w_survive": 1.0}, "roulette"),
    ({"w_min": 0.5, "w_survive": 0.25}, "roulette"),
])
def test_invalid_implicit_capture_rejected(ic, needle):
    p = w.reflective_box([1.0], [[0.5]], [1.0])
    p["implicit_capture"] = ic
    rc, msg = _create(p)
    assert rc == -1 and needle in msg, (rc, msg)
    p = w.reflective_box([1.0], [[0.5]], [1.0], fission=_fis(0.1, 2.0, 1.0))
    p["implicit_capture"] = {"w_min": 0.25, "w_survive": 1.0}
    rc, msg = _create(p)
    assert rc == -1 and "fission" in msg, (rc, msg)


def test_invalid_pins_rejected():
    p = w.pin_lattice(n=1, radius=0.63)                     # wider than half the 1.26 pitch
    rc, msg = _create(p)
    assert rc == -1 and "fit" in msg, (rc, msg)
    p = w.pin_lattice(n=2)
    p["pins"]["material"] = np.full((1, 2, 2), 7, dtype=np.int32)
    rc, msg = _create(p)
    assert rc == -1 and "pin material" in msg, (rc, msg)
    p = w.cfg2_slab_pulse()                                 # y is not a finite axis
    p["pins"] = {"radius": np.array([[[0.1] * 50]]), "material": np.zeros((1, 1, 50), dtype=np.int32)}
    rc, msg = _create(p)
    assert rc == -1 and "finite" in msg, (rc, msg)


def test_invalid_time_crossing_flag_rejected():
    from paper_2305_07636_amd import _binding as b

    d, keep = b.make_desc(w.cfg2_slab_pulse())
    d.time_crossing = 2
    h = C.c_void_p()
    rc = b.lib().mcdc_problem_create(C.byref(d), C.byref(h))
    assert rc == -1 and "time_crossing" in b.lib().mcdc_last_error().decode()


def test_missing_library_fails_loudly(tmp_path):
    """Without the built HIP library the binding raises instead of falling
    back to any CPU path (a fresh interpreter, so the loaded library of this
    session is not reused)."""
    import subprocess
    import sys

    code = ("import paper_2305_07636_amd._binding as b\n"
            f"b.LIB_PATH = {str(tmp_path / 'absent.so')!r}\n"
            "try:\n"
            "    b.lib()\n"
            "except ImportError as e:\n"
            "    print('raised', e)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert "raised" in r.stdout and "is not built" in r.stdout, (r.stdout, r.stderr)


def test_union_grid_beyond_32bit_cell_count_refused():
    """A grid of 2047 x 2047 x 600 union cells (2.5e9 > 2^31 - 1) passes the
    per-axis limits but its cell indices do not fit the device's 32-bit
    tables: it is refused with MCDC_E_UNSUPPORTED before the per-cell tables
    (tens of GB) are built or anything reaches a device."""
    p = w.reflective_box([1.0], [[0.5]], [1.0], size=(20.47, 20.47, 6.0))
    p["tally"]["mesh"] = [np.linspace(0.0, 20.47, 2048), np.linspace(0.0, 20.47, 2048),
                          np.linspace(0.0, 6.0, 601)]
    rc, msg = _create(p)
    assert rc == -5 and "2^31" in msg, (rc, msg)
    # one z-cell fewer than the bound along each axis is still accepted by the
    # per-axis check: 2047 x 2047 x 1 cells compiles past the cell bound
    # (it is the 32-bit product, not an axis, that is refused)
    p["tally"]["mesh"][2] = np.array([0.0, 6.0])
    rc, msg = _create(p)
    assert "2^31" not in msg, (rc, msg)


def test_invalid_moving_plane_rejected():
    p = w.rod_beam_box()
    p["rod"]["z"] = np.array([10.0, np.inf, 0.0])
    rc, msg = _create(p)
    assert rc == -1 and "rod_z" in msg, (rc, msg)
    p = w.rod_beam_box()
    p["rod"]["material"] = np.full((1, 1, 1), 9, dtype=np.int32)
    rc, msg = _create(p)
    assert rc == -1 and "rod material" in msg, (rc, msg)
    p = w.cfg2_slab_pulse()                        # z is not a finite axis
    p["rod"] = {"z": np.zeros(101), "material": np.zeros((1, 1, 1), dtype=np.int32)}
    rc, msg = _create(p)
    assert rc == -1 and "finite z" in msg, (rc, msg)
