"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/pbpqlp.h declares, and rejects bad arguments
synchronously, before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2103_07245_amd import pbpqlp as B

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "pbpqlp.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pbpqlp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = B.library()
    names = _declared_functions()
    assert "pbpqlp_factor" in names and len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name


def test_version_and_status_strings():
    lib = B.library()
    assert lib.pbpqlp_version() == 100
    for s in range(5):
        assert lib.pbpqlp_status_string(s).startswith(b"PBPQLP")


def test_status_flags_match_header():
    text = open(HEADER).read()
    flags = dict((k, int(v)) for k, v in re.findall(r"#define PBPQLP_FLAG_([A-Z]+)\s+(\d+)", text))
    assert flags == {"DEPENDENT": B.FLAG_DEPENDENT, "NONFINITE": B.FLAG_NONFINITE, "INTERNAL": B.FLAG_INTERNAL,
                     "BADINPUT": B.FLAG_BADINPUT}
    # distinct single bits
    assert sorted(flags.values()) == [1, 2, 4, 8]


def test_info_struct_layout():
    assert ctypes.sizeof(B.InfoStruct) == 56
    assert ctypes.sizeof(B.Opts) == 48


FAKE = ctypes.c_void_p(0x1000)


def _factor(m=100, n=80, lda=80, dt=B.F32, k=5, p=3, q=1, ldq=8, ldl=8, ldp=8, opts=None):
    lib = B.library()
    return lib.pbpqlp_factor(FAKE, m, n, lda, dt, k, p, q, ctypes.c_uint64(1), ctypes.c_void_p(0x2000),
                             ldq, ctypes.c_void_p(0x3000), ldl, ctypes.c_void_p(0x4000), ldp,
                             opts, None, None)


@pytest.mark.parametrize("kw", [dict(k=0), dict(p=-1), dict(k=80, p=1), dict(q=17), dict(q=-1),
                                dict(lda=79), dict(ldq=7), dict(ldl=7), dict(ldp=7), dict(m=0),
                                dict(dt=7)])
def test_invalid_arguments_rejected_before_launch(kw):
    assert _factor(**kw) == B.EINVAL


def test_unsupported_width_and_precision():
    # sketches up to 16384 columns are supported (wider ones are blocked by 256)
    assert _factor(m=20000, n=20000, lda=20000, k=16380, p=10, ldq=16390, ldl=16390, ldp=16390) == B.EUNSUPPORTED
    o = B.make_opts("bf16")
    assert _factor(dt=B.F64, opts=ctypes.byref(o)) == B.EUNSUPPORTED


def test_null_pointers_rejected():
    lib = B.library()
    st = lib.pbpqlp_factor(None, 10, 10, 10, B.F32, 2, 1, 0, ctypes.c_uint64(1), FAKE, 3, FAKE, 3,
                           FAKE, 3, None, None, None)
    assert st == B.EINVAL


def test_workspace_size_grows_with_problem():
    a = B.workspace_size(1000, 800, 20, 5)
    b = B.workspace_size(4000, 800, 20, 5)
    c = B.workspace_size(4000, 800, 60, 4)
    assert 0 < a < b < c
    # mixed precision needs the 16-bit operand copies
    assert B.workspace_size(1000, 800, 20, 5, plan="mixed") > a


def test_too_small_workspace_rejected():
    o = B.make_opts("native")
    o.workspace = 0x10000
    o.workspace_bytes = 1024
    assert _factor(opts=ctypes.byref(o)) == B.ENOMEM


def test_problem_struct_layout():
    assert ctypes.sizeof(B.ProblemStruct) == 112


def _problem(**kw):
    pr = B.ProblemStruct()
    pr.A = 0x1000; pr.m = 100; pr.n = 80; pr.lda = 80; pr.k = 5; pr.p = 3; pr.q = 1; pr.seed = 1
    pr.Q = 0x2000; pr.ldq = 8; pr.L = 0x3000; pr.ldl = 8; pr.P = 0x4000; pr.ldp = 8; pr.info = None
    for key, val in kw.items():
        setattr(pr, key, val)
    return pr


@pytest.mark.parametrize("kw", [dict(k=0), dict(lda=79), dict(ldq=7), dict(q=17), dict(A=None)])
def test_batch_rejects_bad_problems_before_allocating(kw):
    lib = B.library()
    probs = (B.ProblemStruct * 3)(_problem(), _problem(**kw), _problem())
    h = ctypes.c_void_p()
    assert lib.pbpqlp_batch_create(3, probs, B.F32, None, ctypes.byref(h)) == B.EINVAL
    assert not h.value


def test_batch_rejects_empty():
    lib = B.library()
    h = ctypes.c_void_p()
    assert lib.pbpqlp_batch_create(0, None, B.F32, None, ctypes.byref(h)) == B.EINVAL


def test_auto_result_layout():
    assert ctypes.sizeof(B.AutoResult) == 40


def test_model_file_errors_before_any_device_work(tmp_path):
    lib = B.library()
    h = ctypes.c_void_p()
    assert lib.pbpqlp_model_load(os.fsencode(str(tmp_path / "missing.bin")), ctypes.byref(h)) == B.EINVAL
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"NOTAMODEL" + bytes(64))
    assert lib.pbpqlp_model_load(os.fsencode(str(bad)), ctypes.byref(h)) == B.EINVAL
    # right magic, wrong dimensions
    import struct
    wrong = tmp_path / "wrong.bin"
    wrong.write_bytes(b"PBQMLP01" + struct.pack("<4iq", 32, 128, 6, 0, 0))
    assert lib.pbpqlp_model_load(os.fsencode(str(wrong)), ctypes.byref(h)) == B.EINVAL
    # truncated parameters
    short = tmp_path / "short.bin"
    short.write_bytes(b"PBQMLP01" + struct.pack("<4iq", 64, 128, 6, 0, 0) + bytes(1000))
    assert lib.pbpqlp_model_load(os.fsencode(str(short)), ctypes.byref(h)) == B.EINVAL


def test_learned_entry_points_reject_null_arguments():
    lib = B.library()
    assert lib.pbpqlp_model_create(None, None) == B.EINVAL
    assert lib.pbpqlp_probe_features(None, 64, None, None) == B.EINVAL
    assert lib.pbpqlp_mlp_forward(None, None, 64, 1, None, 6, None) == B.EINVAL
    assert lib.pbpqlp_mlp_loss_grad(None, None, 64, None, None, 1, None, None, None) == B.EINVAL
    assert lib.pbpqlp_mlp_adam_step(None, 1e-3, None) == B.EINVAL
    res = B.AutoResult()
    assert lib.pbpqlp_factor_auto(None, None, 1000, 1000, 1000, B.F32, 8, 1, 56, 0.1, None, 64,
                                  None, 64, None, 64, None, None, ctypes.byref(res), None) == B.EINVAL
    assert B.MLP_PARAMS == 64 * 128 + 128 + 128 * 128 + 128 + 6 * 128 + 6


def test_tune_cache_file_roundtrip(tmp_path):
    B.tune_clear()
    assert B.tune_lookup(1000, 800, 20, 5) is None
    path = tmp_path / "tune.txt"
    # two classes written by hand in the documented format
    path.write_text("# pbpqlp autotune v1: dt sketch power proj lp32 log2m log2n batched split_k gram_wg ms\n"
                    "1 0 0 0 32 10 10 0 4 256 1.25\n"
                    "1 0 0 0 32 10 10 1 1 16 3.5\n")
    B.tune_load(path)
    # 1000 -> ceil(log2) = 10, 800 -> 10; l = 25 -> lp32 = 32
    assert B.tune_lookup(1000, 800, 20, 5) == {"split_k": 4, "gram_wg": 256, "ms": 1.25}
    assert B.tune_lookup(1000, 800, 20, 5, batched=True)["gram_wg"] == 16
    assert B.tune_lookup(1025, 800, 20, 5) is None          # next size bucket
    assert B.tune_lookup(1000, 800, 20, 5, plan="bf16") is None
    out = tmp_path / "again.txt"
    B.tune_save(out)
    B.tune_clear()
    assert B.tune_lookup(1000, 800, 20, 5) is None
    B.tune_load(out)
    assert B.tune_lookup(1000, 800, 20, 5)["split_k"] == 4
    B.tune_clear()


def test_tune_load_rejects_malformed_files(tmp_path):
    bad = tmp_path / "bad.txt"
    bad.write_text("not a tune file\n")
    with pytest.raises(B.PbpqlpError):
        B.tune_load(bad)
    bad.write_text("# pbpqlp autotune v1\n1 0 0 0 32 10\n")
    with pytest.raises(B.PbpqlpError):
        B.tune_load(bad)
    with pytest.raises(B.PbpqlpError):
        B.tune_load(tmp_path / "missing.txt")
    B.tune_clear()


def test_noalloc_rejects_oversized_problem_before_the_device():
    """pbpqlp_factor_noalloc checks the problem's workspace against its static
    array (PBPQLP_NOALLOC_SCRATCH_BYTES) before any device call: a 16384^2
    problem with l = 256 is refused here, on a host without a GPU."""
    text = open(HEADER).read()
    assert re.search(r"#define PBPQLP_NOALLOC_SCRATCH_BYTES \(64ull << 20\)", text)
    assert B.NOALLOC_SCRATCH_BYTES == 64 << 20
    lib = B.library()
    need = ctypes.c_size_t(0)
    assert lib.pbpqlp_workspace_size(16384, 16384, 200, 56, B.F32, None, ctypes.byref(need)) == B.OK
    assert need.value > B.NOALLOC_SCRATCH_BYTES
    st = lib.pbpqlp_factor_noalloc(FAKE, 16384, 16384, 16384, B.F32, 200, 56, 1, ctypes.c_uint64(1),
                                   ctypes.c_void_p(0x2000), 256, ctypes.c_void_p(0x3000), 256,
                                   ctypes.c_void_p(0x4000), 256, None, None, None)
    assert st == B.EUNSUPPORTED
    # argument errors come first, as for pbpqlp_factor
    st = lib.pbpqlp_factor_noalloc(FAKE, 100, 80, 80, B.F32, 0, 3, 1, ctypes.c_uint64(1),
                                   ctypes.c_void_p(0x2000), 8, ctypes.c_void_p(0x3000), 8,
                                   ctypes.c_void_p(0x4000), 8, None, None, None)
    assert st == B.EINVAL


def test_factor_rr_argument_errors():
    """pbpqlp_factor_rr rejects a missing options record, an unknown
    orientation, a short or aliased R and a negative or NaN rank threshold
    before touching the device; the orientation constants match the header."""
    text = open(HEADER).read()
    consts = dict((k, int(v)) for k, v in re.findall(r"#define PBPQLP_ORIENT_([A-Z]+) (\d+)", text))
    assert consts == {"AT": B.ORIENT["AT"], "A": B.ORIENT["A"], "AUTO": B.ORIENT["auto"]}
    assert ctypes.sizeof(B.RRStruct) == 40
    lib = B.library()

    def call(rr):
        return lib.pbpqlp_factor_rr(FAKE, 100, 80, 80, B.F32, 5, 3, 1, ctypes.c_uint64(1), ctypes.c_void_p(0x2000),
                                    8, ctypes.c_void_p(0x3000), 8, ctypes.c_void_p(0x4000), 8, None,
                                    rr, None, None)

    assert call(None) == B.EINVAL
    for kw in (dict(orientation=3), dict(orientation=-1), dict(R=0x5000, ldr=7), dict(R=0x3000, ldr=8),
               dict(R=0x5004, ldr=8), dict(d_rank=0x6000, rank_tol=-1.0),
               dict(d_rank=0x6000, rank_tol=float("nan"))):
        rr = B.RRStruct()
        for f, v in kw.items():
            setattr(rr, f, v)
        assert call(ctypes.byref(rr)) == B.EINVAL, kw


def test_factor_host_argument_errors():
    """pbpqlp_factor_host rejects null pointers, a negative panel size, short
    leading dimensions, widths beyond the library's limit and misaligned
    outputs before it creates a stream or touches the device; its workspace
    includes the two staging panels."""
    lib = B.library()

    def call(A=FAKE, m=100, n=80, lda=80, k=5, p=3, panel=0, ldq=8, Q=0x2000, P=0x4000):
        return lib.pbpqlp_factor_host(A, m, n, lda, B.F32, k, p, 1, ctypes.c_uint64(1), panel,
                                      ctypes.c_void_p(Q), ldq, ctypes.c_void_p(0x3000), 8,
                                      ctypes.c_void_p(P), 8, None, None, None)

    assert call(A=None) == B.EINVAL
    assert call(panel=-1) == B.EINVAL
    assert call(lda=79) == B.EINVAL
    assert call(ldq=7) == B.EINVAL
    assert call(Q=0x2002) == B.EINVAL
    assert call(Q=0x2000, P=0x2000) == B.EINVAL
    assert call(m=20000, n=20000, lda=20000, k=16380, p=10, ldq=16390) == B.EUNSUPPORTED
    one = B.workspace_size_host(4096, 1024, 40, 8, panel_rows=4096)
    four = B.workspace_size_host(4096, 1024, 40, 8, panel_rows=1024)
    # two staging panels of 4096 (one panel) or 1024 rows of 1024 FP32 values
    assert one - four >= 2 * (4096 - 1024) * 1024 * 4 - (1 << 20)
    assert B.workspace_size_host(4096, 1024, 40, 8, panel_rows=1000) == four   # rounded up to 1024


def test_factor_csr_argument_errors():
    """pbpqlp_factor_csr rejects null arrays, nnz < 0, short leading
    dimensions and reduced-precision plans before touching the device."""
    lib = B.library()

    def call(rowptr=0x1000, colind=0x2000, vals=0x3000, m=100, n=80, nnz=500, k=5, p=3, ldq=8, opts=None):
        return lib.pbpqlp_factor_csr(ctypes.c_void_p(rowptr), ctypes.c_void_p(colind), ctypes.c_void_p(vals), m, n,
                                     nnz, B.F32, k, p, 1, ctypes.c_uint64(1), ctypes.c_void_p(0x4000), ldq,
                                     ctypes.c_void_p(0x5000), 8, ctypes.c_void_p(0x6000), 8, opts, None, None)

    assert call(rowptr=0) == B.EINVAL
    assert call(colind=0) == B.EINVAL
    assert call(nnz=-1) == B.EINVAL
    assert call(ldq=7) == B.EINVAL
    assert call(rowptr=0x1004) == B.EINVAL
    o = B.make_opts("mixed")
    assert call(opts=ctypes.byref(o)) == B.EUNSUPPORTED
    sz = ctypes.c_size_t(0)
    oo = B.make_opts("native")
    assert lib.pbpqlp_workspace_size_csr(4000, 3000, 10 ** 6, 40, 8, B.F32, ctypes.byref(oo), ctypes.byref(sz)) == 0
    # the CSR of A^T (indices and values) and its counters are part of the workspace
    assert sz.value >= 10 ** 6 * 8
