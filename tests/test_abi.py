"""C ABI checks that need no GPU: the library loads, exports every entry point that
include/raspen.h declares, and its host-only partition / validation logic agrees
with the oracle's partition of Section 4.2."""
import ctypes
import os
import re

import pytest

import synth
from oracle.schwarz import partition as oracle_partition

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "raspen.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(rsp_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def R():
    from paper_2411_00546_amd import raspen
    raspen.load()
    return raspen


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ["rsp_solve", "rsp_eval", "rsp_jac_apply", "rsp_local_solve", "rsp_local_residual",
                 "rsp_restrict", "rsp_prolong", "rsp_residual", "rsp_control", "rsp_partition",
                 "rsp_workspace_bytes", "rsp_context_create", "rsp_context_destroy", "rsp_setup",
                 "rsp_version", "rsp_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol(R):
    lib = ctypes.CDLL(R.LIB_PATH)
    bound = {name for name, _, _ in R.SIGNATURES}
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in bound, name           # the binding covers every declaration
        assert hasattr(R, name), name        # and exposes it under the same name


def test_version(R):
    assert R.rsp_version() == 100


@pytest.mark.parametrize("nx,ny,sx,sy,ov", [(63, 63, 2, 2, 2), (255, 255, 8, 8, 4),
                                             (511, 511, 16, 16, 4), (23, 17, 3, 2, 2),
                                             (20, 9, 4, 1, 3), (127, 63, 4, 2, 4), (5, 5, 1, 1, 0)])
def test_partition_matches_oracle(R, nx, ny, sx, sy, ov):
    prob = synth.Problem(nx=nx, ny=ny, sx=sx, sy=sy, overlap=ov)
    S, txm, tym, boxes = R.rsp_partition(R.make_problem(prob))
    subs = oracle_partition(nx, ny, sx, sy, ov)
    assert S == len(subs)
    for b, s in zip(boxes, subs):
        assert tuple(b[:4]) == s.box and tuple(b[4:]) == s.core
    assert txm == max(s.box[1] - s.box[0] for s in subs)
    assert tym == max(s.box[3] - s.box[2] for s in subs)


@pytest.mark.parametrize("change", [dict(sx=4, nx=9), dict(nu=0.0), dict(mu=-1.0), dict(eps_min=0.0),
                                    dict(eps0=1e-9, eps_min=1e-8), dict(gamma=1.0), dict(overlap=-1),
                                    dict(nx=200, sx=2, overlap=4), dict(phi=7)])
def test_invalid_problems_are_rejected(R, change):
    prob = synth.Problem(nx=31, ny=31, sx=2, sy=2, overlap=2)
    for k, v in change.items():
        setattr(prob, k, v)
    with pytest.raises(R.RaspenError) as e:
        R.rsp_partition(R.make_problem(prob))
    assert e.value.code == R.RSP_EINVAL
    assert R.rsp_last_error() != ""


def test_workspace_bytes(R):
    o = R.make_options(synth.Options())
    small = R.rsp_workspace_bytes(R.make_problem(synth.config_small()), o)
    plain = R.rsp_workspace_bytes(R.make_problem(synth.config_plain()), o)
    prec = R.rsp_workspace_bytes(R.make_problem(synth.config_precision()), o)
    assert 0 < small < plain < prec
    # factors dominate: S * tym * M^2 doubles for the 255x255 workload (64 * 40 * 80^2 * 8 B)
    assert plain > 64 * 40 * 80 * 80 * 8
    bad = synth.Problem(nx=9, ny=9, sx=4, sy=1)
    assert R.rsp_workspace_bytes(R.make_problem(bad), o) == 0
    # FP32 line factors take half the factor bytes
    mixed = R.rsp_workspace_bytes(R.make_problem(synth.config_plain()), R.make_options(synth.Options(precision=1)))
    assert plain - mixed == 64 * 40 * 80 * 80 * 4


def test_batch_workspace_bytes(R):
    o = R.make_options(synth.Options())
    a = R.make_problem(synth.config_small())
    b = R.make_problem(synth.config_plain())
    one = R.rsp_batch_workspace_bytes([a], o)
    assert one == R.rsp_workspace_bytes(a, o)
    both = R.rsp_batch_workspace_bytes([a, b], o)
    assert both > R.rsp_workspace_bytes(b, o) > one
    bad = R.make_problem(synth.Problem(nx=9, ny=9, sx=4, sy=1))
    assert R.rsp_batch_workspace_bytes([a, bad], o) == 0
    assert R.rsp_batch_workspace_bytes([], o) == 0


def test_server_and_batch_entry_points_are_declared():
    names = declared_functions()
    for must in ["rsp_solve_batch", "rsp_solve_newton_ras", "rsp_solve_newton", "rsp_batch_workspace_bytes", "rsp_server_create",
                 "rsp_server_submit",
                 "rsp_server_poll", "rsp_server_wait", "rsp_server_stats", "rsp_server_destroy"]:
        assert must in names


def test_tuning_entry_points_are_declared():
    names = declared_functions()
    for must in ["rsp_get_tuning", "rsp_set_tuning", "rsp_autotune", "rsp_set_profiling_filter",
                 "rsp_set_profiling_sample"]:
        assert must in names


def test_struct_layouts_match_the_header(R, tmp_path):
    """The binding's ctypes structs have the sizes and field offsets of the C structs,
    as a plain C compile of the header reports them."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("no C compiler or HIP headers")
    structs = {"rsp_problem": R.rsp_problem, "rsp_options": R.rsp_options, "rsp_history": R.rsp_history,
               "rsp_tuning": R.rsp_tuning, "rsp_server_options": R.rsp_server_options,
               "rsp_server_report": R.rsp_server_report, "rsp_kernel_stat": R.rsp_kernel_stat}
    lines = []
    for name, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for field, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, field, name, field))
    src = tmp_path / "probe.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"raspen.h\"\n"
                   "int main(void) {\n" + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "probe"
    subprocess.run([cc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I",
                    "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(out[name]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(out[name + "." + field]) == getattr(cls, field).offset, (name, field)


def test_bench_and_entry_scripts_parse():
    """bench.py and __graft_entry__.py compile, and bench.py's argument parser runs
    (no GPU needed: --help exits before anything is loaded)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for f in ("bench.py", "__graft_entry__.py"):
        path = os.path.join(root, f)
        with open(path) as fh:
            compile(fh.read(), path, "exec")
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    for flag in ("--method", "--time-every", "--workload", "--gpus", "--steps", "--warmup"):
        assert flag in r.stdout
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
