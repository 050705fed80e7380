"""The host rasterizer (csrc/geometry.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

tests/sanitize/rasterize_driver.cpp and geometry.cpp are built with g++
-fsanitize=address,undefined (host code only: nothing here is GPU code).
Every geometry of the host rasterizer checks, plus the rejected inputs, runs
through the instrumented build; a sanitizer report fails the test, and the
instrumented result must equal what the library's own lq_rasterize gives.
"""
import ctypes as C
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from paper_1911_07045_amd import lqfire

import test_abi_host

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "sanitize", "rasterize_driver.cpp")
GEOMETRY = os.path.join(ROOT, "paper_1911_07045_amd", "csrc", "geometry.cpp")
ENV = dict(os.environ,
           ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1:verify_asan_link_order=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    exe = str(tmp_path_factory.mktemp("asan") / "rasterize_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1911_07045_amd", "csrc"), DRIVER, GEOMETRY, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def _input(shape, periodic, objs, recs, osites):
    p = lqfire.make_params(shape, periodic)
    o, no = lqfire.make_objects(list(objs))
    r, nr = lqfire.make_records(list(recs))
    os_ = np.ascontiguousarray(np.asarray(osites, dtype=np.int64).reshape(-1))
    return (bytes(p) + struct.pack("<i", no) + bytes(o)[:no * C.sizeof(lqfire.Object)]
            + struct.pack("<q", nr) + bytes(r)[:nr * C.sizeof(lqfire.SiteAnchor)]
            + struct.pack("<q", len(os_)) + os_.tobytes())


def _run(exe, data):
    r = subprocess.run([exe], input=data, capture_output=True, env=ENV, timeout=300)
    err = r.stderr.decode(errors="replace")
    assert r.returncode == 0, err
    assert "runtime error" not in err and "Sanitizer" not in err, err
    out = r.stdout
    rc = struct.unpack_from("<i", out, 0)[0]
    if rc != 0:
        return rc, None
    off = 4
    N, n_sim = struct.unpack_from("<qq", out, off)
    off += 16
    types = np.frombuffer(out, np.uint8, N, off)
    off += 2 * N  # types, then the neighbour masks
    n_anch = struct.unpack_from("<q", out, off)[0]
    off += 8
    sites = np.frombuffer(out, np.int64, n_anch, off)
    off += 8 * n_anch
    data = np.frombuffer(out, np.float64, n_anch * lqfire.ANCH_STRIDE, off).reshape(n_anch, -1)
    assert off + data.nbytes == len(out)
    return rc, (types, sites, data, n_sim)


@pytest.mark.parametrize("name", sorted(test_abi_host.GEOMS))
def test_rasterizer_is_clean_under_sanitizers(driver, name):
    shape, periodic, objs, recs, osites = test_abi_host.GEOMS[name]()
    rc, res = _run(driver, _input(shape, periodic, objs, recs, osites))
    assert rc == 0
    types, sites, data, n_sim = res
    t_l, s_l, d_l = lqfire.rasterize(shape, periodic, objs, recs, osites)
    assert np.array_equal(types, t_l)
    assert np.array_equal(sites, s_l)
    assert np.array_equal(data, d_l)
    assert n_sim == int((t_l != 2).sum())


BAD = {
    "sphere_radius_zero": ((8, 8, 8), (True,) * 3,
                           [dict(kind="sphere", center=(4, 4, 4), radius=0.0, law="rp", W=1.0)], (), ()),
    "wall_plane_out_of_range": ((8, 8, 8), (True,) * 3,
                                [dict(kind="wall", axis=2, plane=8, law="nd", W=1.0, dir=(1, 0, 0))], (), ()),
    "record_out_of_range": ((4, 4, 4), (True,) * 3, [],
                            [dict(site=64, law="nd", W=1.0, n0=(1, 0, 0))], ()),
    "record_at_object_site": ((4, 4, 4), (True,) * 3, [],
                              [dict(site=5, law="nd", W=1.0, n0=(1, 0, 0))], (5,)),
    "object_site_negative": ((4, 4, 4), (True,) * 3, [], (), (-1,)),
}


@pytest.mark.parametrize("name", sorted(BAD))
def test_rejected_geometries_are_clean_under_sanitizers(driver, name):
    shape, periodic, objs, recs, osites = BAD[name]
    rc, _ = _run(driver, _input(shape, periodic, objs, recs, osites))
    assert rc == lqfire.LQ_EINVAL
    with pytest.raises(lqfire.LQError) as e:
        lqfire.rasterize(shape, periodic, objs, recs, osites)
    assert e.value.code == lqfire.LQ_EINVAL
