"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function that include/rmrt.h declares, and its parameter derivation
(weights, rates, second-order block) agrees with the independent oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import rmrt_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rmrt.h")

rmrt = pytest.importorskip("paper_2206_00366_amd.rmrt", reason="librmrt.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rmrt_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(rmrt.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding covers the same set
    assert set(names) == set(rmrt.EXPORTED)


def test_checked_library_exports_the_same_symbols():
    """librmrt_checked.so (neighbour indices tested in its FP64 kernels) has
    the production library's entry points and reports itself as checked."""
    path = os.path.join(os.path.dirname(rmrt.LIB_PATH), "librmrt_checked.so")
    if not os.path.exists(path):
        pytest.skip("librmrt_checked.so not built")
    lib = ctypes.CDLL(path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.rmrt_checked_build() == 1
    assert rmrt.lib().rmrt_checked_build() == (1 if rmrt.LIB_PATH == path else 0)
    # production build: the check entry points refuse
    if rmrt.LIB_PATH != path:
        n = ctypes.c_uint()
        assert rmrt.lib().rmrt_checked_violations(None, ctypes.byref(n), None) == rmrt.EINVAL


CASES = [
    dict(lattice="Q9", n=(8, 8, 1), dx=(1.0, 0.5, 1.0), nu=0.02, nu_b=0.05),
    dict(lattice="Q9", n=(8, 8, 1), dx=(1.0, 2.0, 1.0), nu=0.1),
    dict(lattice="Q19", n=(4, 4, 4), dx=(1.0, 1.0, 2.0), nu=0.005),
    dict(lattice="Q19", n=(4, 4, 4), dx=(1.0, 0.5, 2.0), nu=0.03, nu_b=0.2),
    dict(lattice="Q27", n=(4, 4, 4), dx=(1.0, 0.5, 2.0), nu=0.05, nu_b=0.01),
    dict(lattice="Q27", n=(4, 4, 4), dx=(1.0, 2.0, 1.0), nu=0.05, w_corner=0.001),
]


@pytest.mark.parametrize("case", [
    dict(lattice="Q27", n=(4, 4, 4), dx=(1.0, 0.5, 2.0), nu=0.05, nu_b=0.1,
         nu_tensor=(0.03, 0.06, 0.04, 0.02, 0.07, 0.05), nu_b_axis=(0.08, 0.05, 0.12)),
    dict(lattice="Q9", n=(8, 8, 1), dx=(1.0, 0.5, 1.0), nu=0.05, nu_tensor=(0.02, -1, -1, 0.09, -1, -1),
         nu_b_axis=(-1.0, 0.3, -1.0), incompressible=True),
])
def test_viscosity_tensor_rates_match_oracle(case):
    m = O.Model(case)
    d = rmrt.derive(rmrt.make_params(**case))
    np.testing.assert_allclose(np.array(d.s_s)[: m.d], m.s_s, atol=1e-14)
    np.testing.assert_allclose(np.array(d.s_b)[: m.d], m.s_b, atol=1e-14)
    np.testing.assert_allclose(np.array(d.s_pair)[: len(m.pairs)], m.s_pair, atol=1e-14)
    Sb = np.array([[d.Sbar2[i][k] for k in range(m.d)] for i in range(m.d)])
    np.testing.assert_allclose(Sb, m.Sbar21, atol=1e-13)


@pytest.mark.parametrize("case", CASES)
def test_derived_parameters_match_oracle(case):
    m = O.Model(case)
    d = rmrt.derive(rmrt.make_params(**case))
    assert d.q == m.q and d.d == m.d
    assert abs(d.cs2 - m.cs2) < 1e-15
    np.testing.assert_allclose(np.array(d.w)[: m.q], m.w, rtol=0, atol=1e-15)
    assert abs(d.s_nu - m.s_ab) < 1e-14
    np.testing.assert_allclose(np.array(d.s_s)[: m.d], m.s_s, atol=1e-14)
    np.testing.assert_allclose(np.array(d.s_b)[: m.d], m.s_b, atol=1e-14)
    Sb = np.array([[d.Sbar2[i][k] for k in range(m.d)] for i in range(m.d)])
    np.testing.assert_allclose(Sb, m.Sbar21, atol=1e-13)
    assert abs(d.s_hi - m.s_hi) < 1e-14


@pytest.mark.parametrize("case", [
    dict(lattice="Q5", equation="NCDE", n=(8, 8, 1), dx=(1.0, 0.5, 1.0), D0=0.01),
    dict(lattice="Q5", equation="NCDE", n=(8, 8, 1), dx=(1.0, 1.0, 1.0), cs2=1.0 / 3.0, D0=0.01),
    dict(lattice="Q7", equation="NCDE", n=(4, 4, 4), dx=(1.0, 0.5, 2.0), D0=0.01, s_hi=1.2),
    dict(lattice="Q7", equation="NCDE", n=(4, 4, 4), dx=(1.0, 1.0, 1.0), D0=0.01),   # w_0 = 0
])
def test_reduced_lattice_weights_match_oracle(case):
    m = O.Model(dict(case, rho0=0.0))
    d = rmrt.derive(rmrt.make_params(**case))
    assert d.q == m.q and d.d == m.d
    assert abs(d.cs2 - m.cs2) < 1e-15
    np.testing.assert_allclose(np.array(d.w)[: m.q], m.w, rtol=0, atol=1e-15)
    assert min(d.w[: m.q]) >= 0.0
    assert abs(d.s_hi - m.s_hi) < 1e-14


def test_population_bytes():
    """q streams of stride ld: the stream size rounded up to 4 KiB below 1 MiB,
    to 64 KiB below 16 MiB and to whole MiB above."""
    p = rmrt.make_params(lattice="Q27", storage="f16dev", n=(10, 20, 30), nu=0.05)
    assert rmrt.population_bytes(p) == 27 * 12288                      # 12000 B -> 3 x 4 KiB
    p = rmrt.make_params(lattice="Q9", storage="f64", n=(10, 20, 1), nu=0.05)
    assert rmrt.population_bytes(p) == 9 * 4096
    p = rmrt.make_params(lattice="Q19", storage="f32dev", n=(256, 256, 128), nu=0.05)
    assert rmrt.population_bytes(p) == 19 * 4 * 256 * 256 * 128        # 32 MiB: no padding
    p = rmrt.make_params(lattice="Q19", storage="f32dev", n=(256, 256, 127), nu=0.05)
    assert rmrt.population_bytes(p) == 19 * (32 << 20)                 # 31.75 MiB -> 32 MiB
    p = rmrt.make_params(lattice="Q27", storage="f32dev", n=(100, 50, 60), nu=0.05)
    assert rmrt.population_bytes(p) == 27 * (1216 << 10)               # 1.14 MiB -> 19 x 64 KiB
    for n in [(7, 5, 3), (97, 89, 83), (300, 200, 100), (1000, 1000, 1)]:
        for st, es in (("f64", 8), ("f32dev", 4), ("f16dev", 2)):
            p = rmrt.make_params(lattice="Q19" if n[2] > 1 else "Q9", storage=st, n=n, nu=0.05)
            q = 19 if n[2] > 1 else 9
            b = rmrt.population_bytes(p)
            assert b % q == 0
            stream = b // q
            N = n[0] * n[1] * n[2]
            assert N * es <= stream < N * es * 1.0625 + 4096
            assert stream % 4096 == 0


@pytest.mark.parametrize("bad", [
    dict(lattice="Q9", n=(8, 8, 2)),                                 # 2D with nz > 1
    dict(lattice="Q9", n=(8, 8, 1), cs2=0.5, dx=(1.0, 0.5, 1.0)),    # cs2 >= c_y^2
    dict(lattice="Q19", n=(4, 4, 4), dx=(1.0, 0.5, 0.5), cs2=0.2),   # negative Q19 weight
    dict(lattice="Q9", n=(8, 8, 1), nu=-0.1),
    dict(lattice="Q9", n=(8, 8, 1), equation="NCDE", D0=0.0),
    dict(lattice="Q9", n=(0, 8, 1)),
    dict(lattice="Q9", n=(8, 8, 1), dx=(0.0, 1.0, 1.0)),
    dict(lattice="Q9", n=(8, 8, 1), nu=0.1, s_hi=2.5),                  # rate outside (0, 2)
    dict(lattice="Q19", n=(4, 4, 4), nu=0.1, nu_b=0.0),
    dict(lattice="Q5", n=(8, 8, 1), nu=0.1),                          # reduced lattices: NCDE only
    dict(lattice="Q7", n=(4, 4, 4), equation="NCDE", D0=0.01, storage="f16dev"),  # w_0 = 0 with FP16
    dict(lattice="Q5", n=(8, 8, 2), equation="NCDE", D0=0.01),
    dict(lattice="Q5", n=(8, 8, 1), equation="NCDE", D0=0.01, cs2=0.6),   # w_0 < 0
    dict(lattice="Q27", n=(4, 4, 4), nu=0.05, w_corner=0.0, storage="f16dev"),
    dict(lattice=5, n=(4, 4, 4), equation="NCDE", D0=0.01),           # unknown lattice
    dict(lattice="Q9", n=(8, 8, 1), equation="NCDE", D0=0.01, incompressible=True),  # He-Luo is NSE only
    dict(lattice="Q9", n=(8, 8, 1), nu=0.05, incompressible=True, rho0=0.0),
    dict(lattice="Q9", n=(8, 8, 1), nu=0.05, gamma0=True),                          # gamma = 0 is NCDE only
    dict(lattice="Q9", n=(8, 8, 1), nu=0.05, diffusive=True),                       # so is the diffusive scaling
    dict(lattice="Q9", n=(8, 8, 1), nu=0.05, nu_tensor=(float("nan"), -1, -1, -1, -1, -1)),
])
def test_invalid_parameters_rejected(bad):
    with pytest.raises(rmrt.RMRTError) as ei:
        rmrt.derive(rmrt.make_params(**bad))
    assert ei.value.code == rmrt.EINVAL
    assert rmrt.lib().rmrt_last_error()


def test_init_argument_errors_need_no_gpu():
    """Argument validation returns RMRT_EINVAL before any device call."""
    p = rmrt.make_params(lattice="Q9", n=(8, 8, 1), pattern="AB")
    ctx = ctypes.c_void_p()
    rc = rmrt.lib().rmrt_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.c_void_p(16), None, None,
                              ctypes.c_void_p(16), None, 0, None)
    assert rc == rmrt.EINVAL  # AB without f1
    assert rmrt.lib().rmrt_step(None, 1, None) == rmrt.EINVAL


def test_batch_configs_within_launch_bound():
    cfgs = rmrt.Batch.configs()
    assert len(cfgs) >= 4
    for threads, tile_nodes, per_cu, persistent, npt in cfgs:
        assert 64 <= threads <= 256 and threads % 64 == 0
        assert npt in (1, 2)
        assert tile_nodes >= npt * threads
        assert persistent in (0, 1)
        assert persistent == 0 or per_cu >= 1
        assert per_cu != 1 or persistent == 1


def test_single_hip_runtime_in_process():
    """The binding loads torch before the library, so only one libamdhip64 is mapped."""
    import subprocess
    import sys
    code = ("import paper_2206_00366_amd.rmrt as r, torch;"
            "m = open('/proc/self/maps').read();"
            "print(len(set(l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l)))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.stdout.strip() == "1", out.stdout + out.stderr


def test_header_is_valid_c(tmp_path):
    """include/rmrt.h compiles as C99 and its declarations link against the library."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    src = tmp_path / "t.c"
    src.write_text('#include "rmrt.h"\n#include <stdio.h>\n'
                   "int main(void) {\n"
                   "  rmrt_params p = {0}; rmrt_derived d;\n"
                   "  p.lattice = RMRT_Q19; p.n[0] = p.n[1] = p.n[2] = 4; p.dx[0] = p.dx[1] = 1; p.dx[2] = 2;\n"
                   "  p.nu = 0.01; p.nu_b = -1; p.cs2 = -1; p.s_hi = -1; p.w_corner = -1;\n"
                   "  int rc = rmrt_derive(&p, &d);\n"
                   "  printf(\"%d %d %.17g\\n\", rc, d.q, d.w[0]);\n"
                   "  return rc;\n}\n")
    exe = tmp_path / "t"
    inc = os.path.join(ROOT, "include")
    libdir = os.path.dirname(rmrt.LIB_PATH)
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", inc, str(src), "-L", libdir, "-lrmrt",
                        f"-Wl,-rpath,{libdir}", "-o", str(exe)], capture_output=True, text=True)
    if r.returncode != 0 and "cannot find -lrmrt" in r.stderr:
        # the library is named librmrt.so: link it by path
        r = subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", inc, str(src), rmrt.LIB_PATH,
                            f"-Wl,-rpath,{libdir}", "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    rc, q, w0 = out.stdout.split()
    m = O.Model(dict(lattice="Q19", n=(4, 4, 4), dx=(1.0, 1.0, 2.0), nu=0.01))
    assert int(q) == 19 and abs(float(w0) - m.w[0]) < 1e-15


@pytest.mark.parametrize("cname,pyname", [("rmrt_params", "Params"), ("rmrt_derived", "Derived")])
def test_struct_layout_matches_header(tmp_path, cname, pyname):
    """The binding's ctypes structure has the header's members in the header's
    order, its size and its field offsets (a member added to one side only
    would shift every later one)."""
    import ctypes
    import re
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    cls = getattr(rmrt, pyname)
    fields = [f[0] for f in cls._fields_]
    hdr = open(os.path.join(ROOT, "include", "rmrt.h")).read()
    decl = hdr[hdr.index(f"typedef struct {cname} {{"):hdr.index(f"}} {cname};")].split("{", 1)[1]
    decl = re.sub(r"/\*.*?\*/|//[^\n]*", "", decl, flags=re.S)
    names = []
    for stmt in filter(None, (t.strip() for t in decl.split(";"))):
        declarators = re.sub(r"^(unsigned|int|double)\s+", "", stmt)
        names += [re.match(r"\w+", d.strip()).group(0) for d in declarators.split(",")]
    assert names == fields, (names, fields)
    body = "".join(f'  printf("%s %zu\\n", "{f}", offsetof({cname}, {f}));\n' for f in fields)
    src = tmp_path / "layout.c"
    src.write_text('#include "rmrt.h"\n#include <stddef.h>\n#include <stdio.h>\nint main(void) {\n'
                   f'  printf("sizeof %zu\\n", sizeof({cname}));\n' + body + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        timeout=60).stdout.splitlines())
    assert int(out["sizeof"]) == ctypes.sizeof(cls)
    for f in fields:
        assert int(out[f]) == getattr(cls, f).offset, f


def test_batch_rejects_mixed_lattices_without_gpu():
    ps = (rmrt.Params * 2)(rmrt.make_params(lattice="Q19", n=(4, 4, 4)), rmrt.make_params(lattice="Q27", n=(4, 4, 4)))
    f0 = (ctypes.c_void_p * 2)(16, 16)
    f1 = (ctypes.c_void_p * 2)(16, 16)
    b = ctypes.c_void_p()
    assert rmrt.lib().rmrt_batch_create(ctypes.byref(b), 2, ps, f0, f1, None, None) == rmrt.EINVAL
    assert b.value is None


def test_domains_beyond_32bit_indexing_are_refused():
    with pytest.raises(rmrt.RMRTError) as ei:
        rmrt.derive(rmrt.make_params(lattice="Q27", n=(1024, 1024, 256), nu=0.05))
    assert ei.value.code == rmrt.EUNSUPPORTED
    rmrt.derive(rmrt.make_params(lattice="Q27", n=(512, 512, 512), nu=0.05))   # 27 * 2^27 < 2^32
