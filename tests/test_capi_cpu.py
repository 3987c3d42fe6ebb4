"""C-ABI checks that need no GPU: the library loads, exports every function that
include/*.h declares, and rejects bad arguments on the host with the documented
status codes (no HIP call is made before validation passes)."""
import ctypes
import glob
import os
import re

import pytest

from paper_2111_13667_amd import tmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(tmm_[a-z_0-9]+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    assert "tmm_rt" in names and "tmm_status_string" in names


@pytest.mark.parametrize("name", declared_functions())
def test_library_exports_declared_symbol(name):
    lib = tmm.library()
    assert hasattr(lib, name), f"{name} declared in include/ but not exported"


def test_version_and_status_strings():
    lib = tmm.library()
    assert re.match(rb"^\d+\.\d+\.\d+$", lib.tmm_version())
    for s in (0, 1, 2, 3, 4, 5):
        assert lib.tmm_status_string(s)
    assert lib.tmm_status_string(3) == b"non-finite input value"


FAKE = 0x1000  # never dereferenced: validation fails before any device access


def args(**kw):
    base = dict(B=2, L=3, n_wl=4, n_theta=5, d=FAKE, nk=FAKE, n_mat=6, dispersive=1, mat=FAKE,
                wl=FAKE, sin_theta=FAKE, cos_theta=FAKE, pol_mask=3, R=FAKE, T=None, r=None, t=None)
    base.update(kw)
    return tmm.TmmRtArgs(**base)


BAD = [
    ("negative B", dict(B=-1)),
    ("negative L", dict(L=-2)),
    ("negative n_wl", dict(n_wl=-1)),
    ("L too large", dict(L=(1 << 20) + 1)),
    ("pol_mask 0", dict(pol_mask=0)),
    ("pol_mask 4", dict(pol_mask=4)),
    ("unknown flag bit", dict(flags=2)),
    ("unknown flag bits with the check", dict(flags=0x81)),
    ("no outputs", dict(R=None)),
    ("n_mat 0", dict(n_mat=0)),
    ("dispersive 2", dict(dispersive=2)),
    ("nk NULL", dict(nk=None)),
    ("wl NULL", dict(wl=None)),
    ("cos NULL", dict(cos_theta=None)),
    ("d NULL", dict(d=None)),
    ("implicit rows missing", dict(mat=None, n_mat=9)),
]


@pytest.mark.parametrize("case", BAD, ids=[c[0] for c in BAD])
def test_invalid_arguments_rejected_on_host(case):
    lib = tmm.library()
    a = args(**case[1])
    st = lib.tmm_rt(ctypes.byref(a), tmm.TMM_F64, None)
    assert st == tmm.TMM_ERR_INVALID_ARG
    assert lib.tmm_last_error()


def test_null_args_and_bad_dtype():
    lib = tmm.library()
    assert lib.tmm_rt(None, tmm.TMM_F64, None) == tmm.TMM_ERR_INVALID_ARG
    a = args()
    assert lib.tmm_rt(ctypes.byref(a), 7, None) == tmm.TMM_ERR_INVALID_ARG


def test_empty_batch_is_a_no_op():
    lib = tmm.library()
    for kw in (dict(B=0), dict(n_wl=0), dict(n_theta=0)):
        a = args(**kw)
        assert lib.tmm_rt(ctypes.byref(a), tmm.TMM_F64, None) == tmm.TMM_OK


def test_ragged_plan_rejects_bad_offsets_on_host():
    from paper_2111_13667_amd import ragged
    import numpy as np
    bad = [
        (np.array([1, 3]), np.array([0, 5]), np.array([0, 1])),      # does not start at 0
        (np.array([0, -1]), np.array([0, 5]), np.array([0, 1])),     # negative layer count
        (np.array([0, 3]), np.array([0, 0]), np.array([0, 1])),      # no wavelength
        (np.array([0, 3]), np.array([0, 5]), np.array([0, 0])),      # no angle
    ]
    for lo, wo, to in bad:
        with pytest.raises(tmm.TmmError) as e:
            ragged.RaggedPlan(lo, wo, to)
        assert e.value.status == tmm.TMM_ERR_INVALID_ARG


def test_surrogate_config_rejected_on_host():
    # every check runs before the first device call, so a CPU-only host sees them
    from paper_2111_13667_amd import surrogate as S
    lib = S._lib()
    good = dict(n_in=30, n_hidden=256, n_layers=2, n_out=256, n_members=2, max_batch=256, seed=1,
                in_shift=0.0, in_scale=1.0, lr=0.0, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0,
                gemm_tile=0)
    for bad in (dict(gemm_tile=4), dict(gemm_tile=-1), dict(n_hidden=200), dict(max_batch=100),
                dict(n_members=0), dict(eps=0.0), dict(beta1=1.0)):
        cfg = S.SurrogateConfig(**{**good, **bad})
        h = ctypes.c_void_p()
        assert lib.tmm_surrogate_create(ctypes.byref(cfg), ctypes.byref(h)) == tmm.TMM_ERR_INVALID_ARG, bad
        assert not h.value


def test_binding_structs_match_the_c_headers(tmp_path):
    # Every struct the ctypes bindings mirror (tmm_rt_args, tmm_ragged_data,
    # tmm_surrogate_config): field names, offsets and total size as the C
    # compiler lays them out from include/*.h, so that a field added to a header
    # cannot go unnoticed by its binding.
    import ctypes
    import shutil
    import subprocess
    from paper_2111_13667_amd import ragged, surrogate, tmm
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    structs = {"tmm_rt_args": tmm.TmmRtArgs, "tmm_ragged_data": ragged.RaggedData,
               "tmm_surrogate_config": surrogate.SurrogateConfig}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "tmm_rt.h"', '#include "tmm_ragged.h"',
             '#include "tmm_surrogate.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'    printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    include = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([gcc, "-std=c11", "-I", include, str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, key, value = line.split()
        got[(cname, key)] = int(value)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
