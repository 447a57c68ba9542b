"""C ABI checks that need no GPU: the library loads, exports every function the
header declares, and rejects bad arguments on the host before any HIP call."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_2502_00243_amd import fpw

LIB = fpw.LIB_PATH

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libfpw.so not built (run __graft_entry__.build())")


def test_exports_every_declared_function():
    names = fpw.header_functions()
    assert {"fpw_plan", "fpw_eval_batch", "fpw_topk", "fpw_eval_fp64", "fpw_debug_bins", "fpw_plan_destroy",
            "fpw_last_error", "fpw_options_default", "fpw_get_plan_info", "fpw_version"} <= set(names)
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    for n in names:
        assert f" T {n}\n" in out, n


def test_library_has_gfx950_code_object():
    # the fat binary embedded in the library names its offload target
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_options_defaults():
    o = fpw.default_options()
    assert (o.n_bins, o.center, o.tref_mode, o.phase, o.stat_scale, o.topk) == (10, 0, 0, 0, 0, 0)
    assert o.inv_alpha2 == 0.0 and o.use_graph == 1 and o.autotune == 0
    assert o.hist_share == 0 and o.baseline_terms == 0 and o.baseline_scale == 1.0 and o.fuse_prepare == 0
    assert fpw.load().fpw_version().decode().startswith("fpw ")


def _good():
    off = np.array([0, 3, 5], dtype=np.int64)
    t = np.array([0.1, 2.0, 7.5, 1.0, 3.0])
    y = np.array([1.0, 2.0, 1.5, 0.0, 0.3])
    dy = np.full(5, 0.1)
    f = np.linspace(0.1, 3.0, 40)
    return off, t, y, dy, f


CASES = [
    ("no curves", dict(offsets=[0]), fpw.EINVAL),
    ("offsets[0] != 0", dict(offsets=[1, 3, 5]), fpw.EINVAL),
    ("empty curve", dict(offsets=[0, 0, 5]), fpw.EINVAL),
    ("dy = 0", dict(dy=[0.1, 0.1, 0.0, 0.1, 0.1]), fpw.EINVAL),
    ("dy < 0", dict(dy=[0.1, -0.1, 0.1, 0.1, 0.1]), fpw.EINVAL),
    ("nan y", dict(y=[1.0, np.nan, 1.5, 0.0, 0.3]), fpw.EINVAL),
    ("inf t", dict(t=[0.1, np.inf, 7.5, 1.0, 3.0]), fpw.EINVAL),
    ("negative t with t_ref 0", dict(t=[-0.1, 2.0, 7.5, 1.0, 3.0]), fpw.EINVAL),
    ("f = 0", dict(freqs=[0.0, 1.0]), fpw.EINVAL),
    ("f < 0", dict(freqs=[-1.0]), fpw.EINVAL),
    ("nan f", dict(freqs=[np.nan]), fpw.EINVAL),
    ("M = 0", dict(n_bins=0), fpw.EINVAL),
    ("M too large", dict(n_bins=fpw.MAX_BINS + 1), fpw.EUNSUPPORTED),
    ("topk > n_freq", dict(freqs=[1.0, 2.0], opts=dict(topk=3)), fpw.EINVAL),
    ("topk too large", dict(opts=dict(topk=fpw.MAX_TOPK + 1)), fpw.EUNSUPPORTED),
    ("negative alpha prior", dict(opts=dict(inv_alpha2=-1.0)), fpw.EINVAL),
    ("nan alpha prior", dict(opts=dict(inv_alpha2=np.nan)), fpw.EINVAL),
    ("t below given t_ref", dict(opts=dict(tref="given", t_ref=0.5)), fpw.EINVAL),
    ("bad phase", dict(opts=dict(phase=7)), fpw.EINVAL),
    ("bad center", dict(opts=dict(center=9)), fpw.EINVAL),
    ("fp32 fold range", dict(t=[0.1, 2.0, 7.5e6, 1.0, 3.0], opts=dict(phase="df32")), fpw.EUNSUPPORTED),
    ("two freqs per lane in df32", dict(opts=dict(phase="df32", freqs_per_lane=2)), fpw.EUNSUPPORTED),
    ("bad waves per group", dict(opts=dict(waves_per_group=3)), fpw.EINVAL),
    ("derived M does not divide", dict(n_bins=12, opts=dict(derived_bins=(5,))), fpw.EINVAL),
    ("derived M not smaller", dict(n_bins=12, opts=dict(derived_bins=(12,))), fpw.EINVAL),
    ("derived M twice", dict(n_bins=12, opts=dict(derived_bins=(6, 6))), fpw.EINVAL),
    ("too many variants", dict(n_bins=40, opts=dict(derived_bins=(5, 10), all_offsets=True)), fpw.EUNSUPPORTED),
    ("two freqs per lane with variants", dict(n_bins=12, opts=dict(derived_bins=(6,), freqs_per_lane=2)), fpw.EUNSUPPORTED),
    ("bad hist share", dict(opts=dict(hist_share=3)), fpw.EINVAL),
    ("negative hist share", dict(opts=dict(hist_share=-2)), fpw.EINVAL),
    ("hist share with other waves per group", dict(opts=dict(hist_share=2, waves_per_group=4)), fpw.EINVAL),
    ("hist share with two freqs per lane", dict(opts=dict(hist_share=2, freqs_per_lane=2)), fpw.EUNSUPPORTED),
    ("bad fuse prepare", dict(opts=dict(fuse_prepare=2)), fpw.EINVAL),
    ("fused pass with variants", dict(n_bins=12, opts=dict(fuse_prepare=1, derived_bins=(6,))), fpw.EUNSUPPORTED),
    ("fused pass with baseline", dict(opts=dict(fuse_prepare=1, baseline_terms=1)), fpw.EUNSUPPORTED),
    ("fused pass with a point source", dict(opts=dict(fuse_prepare=1, point_source=2)), fpw.EUNSUPPORTED),
    ("fused pass with private histograms", dict(opts=dict(fuse_prepare=1, hist_share=1)), fpw.EUNSUPPORTED),
    ("fused pass with two waves", dict(opts=dict(fuse_prepare=1, waves_per_group=2)), fpw.EUNSUPPORTED),
    ("hist share in df32 with variants", dict(n_bins=12, opts=dict(hist_share=4, phase="df32", derived_bins=(6,))),
     fpw.EUNSUPPORTED),
]


@pytest.mark.parametrize("name,change,expect", CASES, ids=[c[0] for c in CASES])
def test_plan_rejects_bad_arguments_on_host(name, change, expect):
    off, t, y, dy, f = _good()
    args = dict(offsets=off, t=t, y=y, dy=dy, freqs=f, n_bins=4)
    opts = change.pop("opts", {}) if "opts" in change else {}
    args.update({k: np.asarray(v) for k, v in change.items() if k != "n_bins"})
    if "n_bins" in change:
        args["n_bins"] = change["n_bins"]
    st, msg = fpw.plan_status(args["offsets"], args["t"], args["y"], args["dy"], args["freqs"], args["n_bins"], **opts)
    assert st == expect, (name, st, msg)
    assert msg


def test_null_pointers_rejected():
    lib = fpw.load()
    h = ctypes.c_void_p()
    st = lib.fpw_plan(ctypes.byref(h), 1, None, None, None, None, 1, None, None, None)
    assert st == fpw.EINVAL
    assert lib.fpw_plan(None, 1, None, None, None, None, 1, None, None, None) == fpw.EINVAL
    assert lib.fpw_eval_batch(None, None, None, None, None) == fpw.EINVAL
    assert lib.fpw_topk(None, None, 1, None, None, None) == fpw.EINVAL
    assert lib.fpw_eval_fp64(None, None, None) == fpw.EINVAL
    assert lib.fpw_debug_bins(None, 0, 0, 0, 1, None, None) == fpw.EINVAL
    assert lib.fpw_get_plan_info(None, None) == fpw.EINVAL
    lib.fpw_plan_destroy(None)  # no-op


def test_valid_plan_without_gpu_reports_hip_error():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    off, t, y, dy, f = _good()
    st, msg = fpw.plan_status(off, t, y, dy, f, 4)
    assert st == fpw.EHIP and msg


# ---------------------------------------------------------------- shared-timestamp plans


def _good_shared():
    t = np.array([0.1, 2.0, 7.5, 9.0])
    y = np.array([[1.0, 2.0, 1.5, 0.0], [0.3, 0.1, -0.2, 0.0], [0.0, 0.5, 0.5, 0.1]])
    dy = np.full(y.shape, 0.1)
    f = np.linspace(0.1, 3.0, 40)
    return t, y, dy, f


SHARED_CASES = [
    ("nan y", dict(y=lambda y: np.where(y == 2.0, np.nan, y)), {}, fpw.EINVAL),
    ("dy = 0", dict(dy=lambda d: np.where(np.arange(d.size).reshape(d.shape) == 5, 0.0, d)), {}, fpw.EINVAL),
    ("negative t", dict(t=lambda t: t - 1.0), {}, fpw.EINVAL),
    ("f = 0", dict(f=lambda f: np.concatenate([[0.0], f])), {}, fpw.EINVAL),
    ("M too large for the matrix kernel", {}, dict(n_bins=65, shared_kernel="matrix"), fpw.EUNSUPPORTED),
    ("df32 on the matrix kernel", {}, dict(phase="df32", shared_kernel="matrix"), fpw.EUNSUPPORTED),
    ("variants on the matrix kernel", {}, dict(n_bins=20, derived_bins=(10,), shared_kernel="matrix"), fpw.EUNSUPPORTED),
    ("bad kernel choice", {}, dict(shared_kernel=3), fpw.EINVAL),
]


@pytest.mark.parametrize("name,change,opts,expect", SHARED_CASES, ids=[c[0] for c in SHARED_CASES])
def test_shared_plan_rejects_bad_arguments_on_host(name, change, opts, expect):
    t, y, dy, f = _good_shared()
    arrs = dict(t=t, y=y, dy=dy, f=f)
    for k, fn in change.items():
        arrs[k] = fn(arrs[k])
    opts = dict(opts)
    n_bins = opts.pop("n_bins", 4)
    st, msg = fpw.plan_shared_status(arrs["t"], arrs["y"], arrs["dy"], arrs["f"], n_bins, **opts)
    assert st == expect, (name, st, msg)
    assert msg


def test_shared_plan_null_and_empty_arguments():
    lib = fpw.load()
    h = ctypes.c_void_p()
    assert lib.fpw_plan_shared(ctypes.byref(h), 1, 1, None, None, None, 1, None, None, None) == fpw.EINVAL
    t, y, dy, f = _good_shared()
    P = ctypes.POINTER(ctypes.c_double)
    args = [t.ctypes.data_as(P), y.ctypes.data_as(P), dy.ctypes.data_as(P), len(f), f.ctypes.data_as(P), None, None]
    assert lib.fpw_plan_shared(ctypes.byref(h), 0, 4, *args) == fpw.EINVAL
    assert lib.fpw_plan_shared(ctypes.byref(h), 3, 0, *args) == fpw.EINVAL
    with pytest.raises(ValueError):
        fpw.plan_shared_status(t, y[:, :3], dy, f, 4)


BASELINE_CASES = [
    ("negative terms", dict(baseline_terms=-1), fpw.EINVAL),
    ("too many terms", dict(baseline_terms=4), fpw.EUNSUPPORTED),
    ("zero scale", dict(baseline_terms=2, baseline_scale=0.0), fpw.EINVAL),
    ("nan scale", dict(baseline_terms=2, baseline_scale=float("nan")), fpw.EINVAL),
    ("df32 phase", dict(baseline_terms=2, phase="df32"), fpw.EUNSUPPORTED),
    ("M too large", dict(baseline_terms=1, n_bins=65), fpw.EUNSUPPORTED),
    ("with derived bins", dict(baseline_terms=1, n_bins=12, derived_bins=(6,)), fpw.EUNSUPPORTED),
]


@pytest.mark.parametrize("name,opts,expect", BASELINE_CASES, ids=[c[0] for c in BASELINE_CASES])
def test_baseline_options_checked_on_host(name, opts, expect):
    off, t, y, dy, f = _good()
    opts = dict(opts)
    n_bins = opts.pop("n_bins", 4)
    st, msg = fpw.plan_status(off, t, y, dy, f, n_bins, **opts)
    assert st == expect, (name, st, msg)
    assert msg


def test_baseline_defaults():
    o = fpw.default_options()
    assert o.baseline_terms == 0 and o.baseline_scale == 1.0 and o.shared_kernel == 0


def _build_c_client(tmp_path):
    import shutil

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    here = os.path.dirname(os.path.abspath(__file__))
    root = os.path.dirname(here)
    libdir = os.path.dirname(LIB)
    exe = str(tmp_path / "abi_check")
    cmd = [cc, "-std=c99", "-Wall", "-Werror", "-O1", os.path.join(here, "c", "abi_check.c"), "-I", os.path.join(root, "include"),
           "-L", libdir, "-l:libfpw.so", f"-Wl,-rpath,{libdir}", "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,/opt/rocm/lib", "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_c_client_compiles_links_and_checks_arguments(tmp_path):
    """The header is plain C; a C program links libfpw and sees the host-side checks."""
    exe = _build_c_client(tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "C ABI checks ok" in r.stdout


@pytest.mark.parametrize("struct", ["fpw_options", "fpw_plan_info"])
def test_binding_structs_match_header_layout(tmp_path, struct):
    """The ctypes mirrors of the header's structs have the C compiler's field offsets and size."""
    import shutil

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirror = {"fpw_options": fpw.Options, "fpw_plan_info": fpw.PlanInfo}[struct]
    names = [f[0] for f in mirror._fields_]
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "layout.c"
    body = "".join(f'  printf("{n} %zu\\n", offsetof({struct}, {n}));\n' for n in names)
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"fpw.h\"\nint main(void) {\n"
                   f'  printf("sizeof %zu\\n", sizeof({struct}));\n{body}  return 0;\n}}\n')
    exe = str(tmp_path / "layout")
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", str(src), "-I", os.path.join(root, "include"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = dict(line.split() for line in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n") if line)
    assert int(out["sizeof"]) == ctypes.sizeof(mirror)
    for n in names:
        assert int(out[n]) == getattr(mirror, n).offset, n


def _llvm_tool(name):
    path = os.path.join("/opt/rocm/llvm/bin", name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not found")
    return path


def test_every_registered_kernel_exists_in_the_device_code(tmp_path):
    """The host side registers each kernel (and device variable) under its mangled device name; the
    gfx950 code objects must define every one of them, or the runtime cannot load the library's
    kernels.  (Host and device compilations number unnamed types independently, so a kernel
    signature that mentions one can mangle differently on the two sides.)"""
    objcopy, readelf, bundler = _llvm_tool("llvm-objcopy"), _llvm_tool("llvm-readelf"), _llvm_tool("clang-offload-bundler")
    rodata, fatbin = tmp_path / "rodata.bin", tmp_path / "fatbin.bin"
    subprocess.run([objcopy, "-O", "binary", "--only-section=.rodata", LIB, str(rodata)], check=True)
    subprocess.run([objcopy, "-O", "binary", "--only-section=.hip_fatbin", LIB, str(fatbin)], check=True)
    # names handed to the runtime at registration: mangled fpw symbols among the host's constant strings
    registered = {s.decode() for s in rodata.read_bytes().split(b"\0") if s.startswith(b"_ZN3fpw")}
    assert registered, "no registered kernel names found"
    # device symbols: every offload bundle in the fat binary section, gfx950 part
    blob = fatbin.read_bytes()
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    starts = [i for i in range(len(blob)) if blob.startswith(magic, i)]
    assert starts, "no offload bundles"
    defined = set()
    for n, a in enumerate(starts):
        b = starts[n + 1] if n + 1 < len(starts) else len(blob)
        part, code = tmp_path / f"bundle{n}.bin", tmp_path / f"bundle{n}.co"
        part.write_bytes(blob[a:b])
        subprocess.run([bundler, "--unbundle", "--type=o", f"--input={part}", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                        f"--output={code}"], check=True)
        syms = subprocess.run([readelf, "--dyn-syms", "-W", str(code)], check=True, capture_output=True, text=True).stdout
        defined |= {line.split()[-1] for line in syms.splitlines() if " FUNC " in line or " OBJECT " in line}
    missing = sorted(registered - defined)
    assert not missing, f"{len(missing)} registered kernels have no device code, e.g. {missing[0]}"


# ---------------------------------------------------------------- per-bin sum formats (host-side routing)
def _weights_batch(kind, n=400, C=3):
    rng = np.random.default_rng(7)
    t = np.concatenate([np.sort(rng.uniform(0, 1000, n)) for _ in range(C)])
    if kind == "ordinary":
        dy = 0.02 * np.exp(0.5 * rng.standard_normal(n * C))
    elif kind == "dominant":
        dy = np.full(n * C, 0.02)
        dy[n // 2] = 1e-6  # curve 0: one point 2e4 times more precise
    else:  # errors over nine decades in curve 0: beyond the wide format as well
        dy = np.full(n * C, 0.02)
        dy[:n] = 10.0 ** rng.uniform(-9.0, 0.0, n)
    y = dy * rng.standard_normal(n * C)
    return np.arange(C + 1) * n, t, y, dy, np.linspace(0.1, 5.0, 100)


@pytest.mark.parametrize(
    "kind,opts,expect",
    [
        ("dominant", dict(baseline_terms=2), fpw.EUNSUPPORTED),  # the baseline kernel's sums are 32-bit
        ("dominant", dict(derived_bins=(10,)), fpw.EUNSUPPORTED),  # multi-M reuse needs the narrow words
        ("dominant", dict(phase="df32"), fpw.EUNSUPPORTED),
        ("dominant", dict(phase="fp32"), fpw.EUNSUPPORTED),
        ("dominant", dict(fuse_prepare=1), fpw.EUNSUPPORTED),
        ("dominant", dict(n_bins=157), fpw.EUNSUPPORTED),  # wide histograms: M <= FPW_MAX_WIDE_BINS
        ("beyond", {}, fpw.EUNSUPPORTED),
        ("ordinary", dict(sum_format="wide", baseline_terms=1), fpw.EUNSUPPORTED),
        ("ordinary", dict(sum_format=2), fpw.EINVAL),
        # accepted on the host: these reach the device (no GPU here: a HIP error, never an argument error)
        ("dominant", {}, fpw.EHIP),
        ("dominant", dict(n_bins=156), fpw.EHIP),
        ("ordinary", dict(sum_format="wide"), fpw.EHIP),
        ("ordinary", dict(baseline_terms=2), fpw.EHIP),
    ],
)
def test_sum_formats_routed_on_host(kind, opts, expect):
    off, t, y, dy, f = _weights_batch(kind)
    opts = dict(opts)
    M = opts.pop("n_bins", 20)
    st, msg = fpw.plan_status(off, t, y, dy, f, M, **opts)
    if expect == fpw.EHIP and st in (fpw.EHIP, fpw.ENOMEM):
        return
    assert st == expect, (st, msg)
    assert msg


@pytest.mark.parametrize("dy_bad", [1e-170, 1e160])
def test_weights_must_be_finite_normal_doubles(dy_bad):
    off, t, y, dy, f = _weights_batch("ordinary")
    dy = dy.copy()
    dy[5] = dy_bad
    st, msg = fpw.plan_status(off, t, y, dy, f, 20)
    assert st == fpw.EUNSUPPORTED and "1/dy^2" in msg


def test_shared_plan_with_wide_weights_refuses_the_matrix_kernel():
    off, t, y, dy, f = _weights_batch("dominant", n=300, C=4)
    T = t[:300]
    Y, DY = y.reshape(4, 300), dy.reshape(4, 300)
    st, msg = fpw.plan_shared_status(T, Y, DY, f, 20, shared_kernel="matrix")
    assert st == fpw.EUNSUPPORTED and "30-bit" in msg
