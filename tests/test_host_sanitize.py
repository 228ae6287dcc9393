"""The host side of the library (mesh validation, pattern and plan build,
reference tensors, filter build) compiled from its own sources with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer, run on valid meshes of every
element type (structured, jittered, sheared, renumbered) and on meshes each
refusal path must catch (node out of range, repeated node, inverted element,
a node with more adjacent elements than the plan holds).  Any out-of-bounds
access, use after free, signed overflow or misaligned access aborts the run."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2505_02438_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2505_02438_amd", "csrc")
HOST_SOURCES = ["reference.cpp", "plan.cpp", "soptx.cpp", "filter.cpp", "oc.cpp"]


def _write(path, m):
    cells = np.ascontiguousarray(m.cells, dtype=np.int32)
    coords = np.ascontiguousarray(m.coords, dtype=np.float64)
    with open(path, "wb") as fh:
        fh.write(np.array([m.elem, coords.shape[1]], dtype=np.int32).tobytes())
        fh.write(np.array([coords.shape[0], cells.shape[0]], dtype=np.int64).tobytes())
        fh.write(coords.tobytes())
        fh.write(cells.tobytes())


def _shuffled(m, seed):
    rng = np.random.default_rng(seed)
    pn = rng.permutation(m.n_nodes)
    pe = rng.permutation(m.n_cells)
    coords = np.empty_like(m.coords)
    coords[pn] = m.coords
    return I.Mesh(m.elem, coords, pn[m.cells[pe]].astype(np.int32))


def _cases():
    rng = np.random.default_rng(81)
    star = 33
    ang = 2 * np.pi * np.arange(star) / star
    sc = np.vstack([[0.0, 0.0], np.stack([np.cos(ang), np.sin(ang)], axis=1)])
    stc = np.array([[0, 1 + k, 1 + (k + 1) % star] for k in range(star)], dtype=np.int32)
    hx = I.hex_grid(5, 4, 3)
    bad_idx = I.Mesh(hx.elem, hx.coords, hx.cells.copy())
    bad_idx.cells[3, 2] = hx.n_nodes
    rep = I.Mesh(hx.elem, hx.coords, hx.cells.copy())
    rep.cells[2, 1] = rep.cells[2, 0]
    inv = I.Mesh(hx.elem, hx.coords, hx.cells[:, [1, 0, 3, 2, 5, 4, 7, 6]].copy())
    return {
        # name: (mesh, expected validate status, expected plan status, expected general-plan status)
        "quad": (I.quad_grid(9, 6), 0, 0, 0),
        "tri_jitter": (I.tri_grid(8, 5, jitter=0.2, rng=rng), 0, 0, None),
        "hex": (hx, 0, 0, 0),
        "hex_sheared": (I.skew_mesh(I.hex_grid(4, 3, 3), "global"), 0, 0, 0),
        "hex_shuffled": (_shuffled(I.hex_grid(5, 4, 4), 82), 0, 0, 0),
        "hex_jitter": (I.jitter_interior(I.hex_grid(4, 4, 3), 0.2, rng), -5, -5, 0),
        "tet10": (I.kuhn_p2_tets(3, 2, 2, jitter=0.15, rng=rng), 0, 0, None),
        "tet10_shuffled": (_shuffled(I.kuhn_p2_tets(2, 2, 2), 83), 0, 0, None),
        "hex27": (I.hex27_grid(2, 2, 2), -2, -2, 0),
        "star33": (I.Mesh(I.TRI3, sc, stc), 0, -6, None),
        "bad_index": (bad_idx, -3, -3, -3),
        "repeated_node": (rep, -3, -3, -3),
        "inverted": (inv, -4, -4, -4),
    }


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("sanitize")
    objs = []
    flags = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-pthread"]
    for src in HOST_SOURCES + [os.path.join(ROOT, "tests", "sanitize_host.cpp")]:
        o = str(d / (os.path.basename(src) + ".o"))
        subprocess.check_call([gxx, *flags, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    exe = str(d / "sanitize_host")
    subprocess.check_call([gxx, "-fsanitize=address,undefined", "-pthread", "-o", exe, *objs,
                           "-Wl,--unresolved-symbols=ignore-all"])
    return exe, d


def test_host_sources_clean_under_asan_ubsan(driver):
    exe, d = driver
    cases = _cases()
    files = []
    for name, (m, *_rest) in cases.items():
        f = str(d / f"{name}.mesh")
        _write(f, m)
        files.append(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe, *files], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-6000:]
    lines = {os.path.basename(ln.split(":")[0])[:-5]: ln for ln in res.stdout.splitlines()}
    for name, (m, ev, ep, eg) in cases.items():
        words = lines[name].split()
        got = dict(zip(words[1::2], words[2::2]))
        assert int(got["validate"]) == ev, lines[name]
        assert int(got["plan"]) == ep, lines[name]
        if eg is not None:
            assert int(got["general"]) == eg, lines[name]
        if ev == 0:
            assert int(got["filter"]) == 0 and int(got["reference"]) == 0, lines[name]
