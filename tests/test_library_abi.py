"""The C-ABI library builds, loads and exports every symbol the header
declares; host-side argument checks reject bad calls (no GPU work)."""
import ctypes
import os
import re

import pytest

from paper_2606_05687_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pinmpc.h")).read()
    return sorted(set(re.findall(r"\b(pinmpc_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    lib = binding.load()
    names = _declared()
    assert "pinmpc_solve" in names and "pinmpc_create" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(binding.EXPORTS) <= set(names)


def test_struct_layouts_match_header():
    # field order and C types as declared in include/pinmpc.h
    assert ctypes.sizeof(binding.Settings) == 72
    # batch, n_max, 15 pointers, contacts (int32, padded to 8)
    assert ctypes.sizeof(binding.Batch) == 8 + 15 * 8 + 8
    assert binding.Batch.contacts.offset == 8 + 15 * 8
    assert ctypes.sizeof(binding.Out) == 6 * 8


def test_default_settings_and_errors():
    lib = binding.load()
    s = binding.default_settings()
    assert s.iters == 100 and abs(s.rho - 10.0) < 1e-6 and s.refine == 1
    assert lib.pinmpc_strerror(-3).decode() == "workspace exceeds the HBM budget"
    nb = ctypes.c_size_t()
    assert lib.pinmpc_workspace_bytes(ctypes.byref(s), 4096, 20, ctypes.byref(nb)) == 0
    assert 1e8 < nb.value < 2e9
    assert lib.pinmpc_workspace_bytes(ctypes.byref(s), 16, 0, ctypes.byref(nb)) == -1
    assert lib.pinmpc_workspace_bytes(ctypes.byref(s), 16, binding.NMAX_LONG + 1,
                                      ctypes.byref(nb)) == -1
    assert lib.pinmpc_workspace_bytes(ctypes.byref(s), 16, binding.NMAX_LONG, ctypes.byref(nb)) == 0
    # four contacts per stage (feet and hands): horizons up to NMAX, more bytes
    n2, n4 = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.pinmpc_workspace_bytes_contacts(ctypes.byref(s), 4096, 20, 2, ctypes.byref(n2)) == 0
    assert lib.pinmpc_workspace_bytes(ctypes.byref(s), 4096, 20, ctypes.byref(nb)) == 0
    assert n2.value == nb.value
    assert lib.pinmpc_workspace_bytes_contacts(ctypes.byref(s), 4096, 20, 4, ctypes.byref(n4)) == 0
    assert n4.value > n2.value
    assert lib.pinmpc_workspace_bytes_contacts(ctypes.byref(s), 16, binding.NMAX, 4,
                                               ctypes.byref(n4)) == 0
    for bad_c, n in ((4, binding.NMAX + 1), (3, 10), (1, 10), (-4, 10)):
        assert lib.pinmpc_workspace_bytes_contacts(ctypes.byref(s), 16, n, bad_c,
                                                   ctypes.byref(n4)) == -1, (bad_c, n)
    # null context / null arguments are rejected before any device call
    assert lib.pinmpc_solve(None, None, None, None) == -1
    assert lib.pinmpc_destroy(None) == -1
    h = ctypes.c_void_p()
    bad = binding.default_settings(rho=-1.0)
    assert lib.pinmpc_create(ctypes.byref(h), 0, 0, ctypes.byref(bad)) == -1
    # settings are validated before any device call
    for over in (dict(refine_passes=0, ipm_iters=0), dict(refine_passes=1001),
                 dict(ipm_iters=-1), dict(form=3), dict(form=-2), dict(precision=3),
                 dict(kkt_tol=0.0), dict(group=0), dict(group=3), dict(group=8),
                 dict(scan=1), dict(scan=3), dict(scan=16), dict(scan=-2)):
        bad = binding.default_settings(**over)
        assert lib.pinmpc_create(ctypes.byref(h), 0, 0, ctypes.byref(bad)) == -1, over
        assert lib.pinmpc_workspace_bytes(ctypes.byref(bad), 16, 10, ctypes.byref(nb)) in (0, -1)


def test_stats_ring_matches_header_and_rejects_bad_calls():
    text = open(os.path.join(ROOT, "include", "pinmpc.h")).read()
    ring = int(re.search(r"#define PINMPC_STATS_RING (\d+)", text).group(1))
    assert ring == binding.STATS_RING
    lib = binding.load()
    d = [ctypes.c_double() for _ in range(4)]
    refs = [ctypes.byref(v) for v in d]
    assert lib.pinmpc_stats_back(None, 0, *refs) == -1
    assert lib.pinmpc_stats(None, *refs) == -1


def test_noalloc_constants_match_header_and_null_calls_rejected():
    text = open(os.path.join(ROOT, "include", "pinmpc.h")).read()
    m = re.search(r"#define PINMPC_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == binding.NOALLOC_SCRATCH_BYTES
    assert int(re.search(r"PINMPC_ETOOBIG = (-\d+)", text).group(1)) == binding.E_TOOBIG
    lib = binding.load()
    assert lib.pinmpc_solve_noalloc(None, None, None, None) == -1
    assert b"static scratch" in lib.pinmpc_strerror(binding.E_TOOBIG)


def test_boundary_calls_reject_null_arguments():
    lib = binding.load()
    assert lib.pinmpc_build_dynamics(None, None, None, None, None) == -1
    assert lib.pinmpc_server_export_state(None, 0, 1, None, 0) == -1
    assert lib.pinmpc_server_import_state(None, 0, 1, None, 0) == -1
    assert lib.pinmpc_stats_traffic(None, None, None) == -1
    text = open(os.path.join(ROOT, "include", "pinmpc.h")).read()
    assert int(re.search(r"#define PINMPC_NMAX (\d+)", text).group(1)) == binding.NMAX
    assert int(re.search(r"#define PINMPC_NMAX_LONG (\d+)", text).group(1)) == binding.NMAX_LONG
    assert binding.WARM_SLOT_BYTES == binding.NMAX * 5 * 25 * 4
    assert ctypes.sizeof(binding.Physics) == 16 + 7 * 8


def test_landmark_struct_and_null_store_rejected():
    lib = binding.load()
    assert ctypes.sizeof(binding.Landmarks) == 16 + 2 * 8
    assert lib.pinmpc_landmarks_clear(None, None, None) == -1
    assert lib.pinmpc_landmarks_push(None, 10, None, None, 0, None) == -1
    assert lib.pinmpc_landmark_reward(None, None, 0, None, None, 1.0, None, None, None) == -1
    empty = binding.Landmarks(0, 5, 11, 1, None, None)
    assert lib.pinmpc_landmarks_clear(ctypes.byref(empty), None, None) == 0
