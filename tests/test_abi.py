"""C ABI checks that need no GPU: the library loads, exports every symbol that
include/axs.h declares, the binding's table matches the header, and the
entry points reject bad handles without touching a device."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "axs.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(axs_[a-z_0-9]+)\s*\(", text))
    return names - {"axs_alloc_fn", "axs_free_fn"}


@pytest.fixture(scope="module")
def lib():
    from paper_1406_0236_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.load()


def test_header_declares_the_boundary():
    names = header_functions()
    for f in ("axs_build_body", "axs_precompute_scattering", "axs_apply_matvec", "axs_solve"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1406_0236_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = header_functions() - exported
    assert not missing, missing
    for name in header_functions():
        getattr(lib, name)


def test_binding_table_matches_header():
    from paper_1406_0236_amd import _lib
    assert set(_lib.EXPORTS) == header_functions()


def test_binding_constants_match_header_enums():
    """The precision, solve-mode and status values the binding passes and
    decodes are the ones the header's enums define."""
    from paper_1406_0236_amd import _lib
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    enum = {k: int(v) for k, v in re.findall(r"\b(AXS_[A-Z_0-9]+)\s*=\s*(-?\d+)", text)}
    for name in ("FP32", "FP64", "SOLVE_FP64", "SOLVE_MIXED", "SOLVE_CERTIFY", "SOLVE_UNPRECONDITIONED",
                 "SOLVE_RESTART_INNER"):
        assert getattr(_lib, name) == enum["AXS_" + name], name
    for code, name in _lib._STATUS.items():
        assert enum[name] == code, name
    assert (_lib.AXS_OK, _lib.AXS_NOT_CONVERGED) == (enum["AXS_OK"], enum["AXS_NOT_CONVERGED"])


def test_null_handles_are_rejected(lib):
    assert lib.axs_destroy(None) == -1
    assert lib.axs_last_error(None) == b"null context"
    assert lib.axs_precompute_scattering(None) == -1
    assert lib.axs_apply_matvec(None, None, None, 1, 0) == -1
    n = ctypes.c_int64()
    assert lib.axs_num_unknowns(None, ctypes.byref(n)) == -1


def test_warm_start_entry_points_reject_bad_handles(lib):
    """Training, prediction and the warm-start encoding refuse null handles and a
    missing hyperparameter string before touching a device."""
    n = ctypes.c_int64()
    kr = (ctypes.c_double * 2)(1.0, 2.0)
    assert lib.axs_mlp_train(None, None, None, 1, b'{"k_min": 1, "k_max": 2}', None) == -1
    assert lib.axs_mlp_train(None, None, None, 1, None, None) == -1
    assert lib.axs_mlp_predict(None, None, None, None, 1, kr, None) == -1
    assert lib.axs_warm_start_size(None, 8, ctypes.byref(n)) == -1
    assert lib.axs_warm_start_encode(None, None, None, 1, 8, None) == -1
    assert lib.axs_warm_start_decode(None, None, None, 1, 8, None) == -1
    assert lib.axs_mlp_destroy(None) == -1


def test_create_rejects_bad_arguments(lib):
    from paper_1406_0236_amd import _lib
    h = ctypes.c_void_p()
    # null output handle, and a device index that cannot exist
    assert lib.axs_create(None, 0, None, _lib.ALLOC_FN(0), _lib.FREE_FN(0), None) == -1
    assert lib.axs_create(ctypes.byref(h), 1 << 20, None, _lib.ALLOC_FN(0), _lib.FREE_FN(0), None) == -1
    assert not h.value


def test_product_path_has_no_fallback_when_library_is_missing(monkeypatch, tmp_path):
    from paper_1406_0236_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


def test_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1406_0236_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dp, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", text), f


def test_traffic_figure_belongs_to_the_current_kernel_source():
    """bench.py reports the FP32 inter-body kernel's measured HBM bytes only
    for the kernel source they were taken on; the profile that holds them
    names the same fingerprint, so a change of the kernel's code shows here
    until its counter passes are taken again."""
    import bench
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sha = bench.source_fingerprint(os.path.join(root, "paper_1406_0236_amd", "csrc", "interbody.hip"))
    assert sha == bench.TRAFFIC_SOURCE_SHA
    with open(os.path.join(root, "profiles", "interbody_sphere_lattice_27_k4pi_pmc.md")) as f:
        text = f.read()
    assert f"`{sha}`" in text
    mb = float(re.search(r"\*\*([0-9.]+) MB\*\*", text).group(1))
    assert abs(mb * 1e6 - bench.TRAFFIC_BYTES) < 0.1e6


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU: --gpus 2 exits with status 2 and says so,
    before it imports torch or touches a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2, (r.returncode, r.stderr)
    assert "one GPU only" in r.stderr and r.stdout == ""
