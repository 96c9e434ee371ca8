"""The C ABI without a GPU: the library builds, exports every declared entry
point, its structs have the layout the header states, and argument checks that
run before any device access return the documented codes."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dicodile.h")


@pytest.fixture(scope="module")
def lib():
    import paper_1901_09235_amd as dl
    from paper_1901_09235_amd import build
    if not os.path.exists(dl.library_path()):
        build.build()
    return dl.load()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\w[\w\s\*]*?\b(dicodile_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 8
    out = subprocess.run(["nm", "-D", "--defined-only", lib._name], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (dicodile_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)


def test_struct_layouts_match_header(tmp_path):
    """Compile a plain C probe against the header and compare sizes/offsets
    with the ctypes mirrors of the binding."""
    import paper_1901_09235_amd as dl
    src = tmp_path / "probe.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "dicodile.h"
int main(void) {
  printf("%zu %zu %zu\\n", sizeof(dcdl_shape), sizeof(dcdl_csc_opts), sizeof(dcdl_csc_info));
  printf("%zu %zu %zu %zu\\n", offsetof(dcdl_csc_opts, max_rounds), offsetof(dcdl_csc_opts, kkt_target),
         offsetof(dcdl_csc_info, converged), offsetof(dcdl_csc_info, n_passes));
  printf("%zu %zu %zu %zu\\n", sizeof(dcdl_batch_opts), sizeof(dcdl_batch_info), sizeof(dcdl_csc_info),
         offsetof(dcdl_csc_info, t_worker_apply_s));
  printf("%zu %zu %zu %zu\\n", sizeof(dcdl_server_opts), sizeof(dcdl_server_stats),
         offsetof(dcdl_server_opts, tile), offsetof(dcdl_server_stats, t_busy_s));
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(dcdl_dict_opts), sizeof(dcdl_dict_info), sizeof(dcdl_cdl_opts),
         sizeof(dcdl_cdl_info), offsetof(dcdl_cdl_opts, dict), offsetof(dcdl_cdl_info, n_updates));
  printf("%zu %zu\\n", sizeof(dcdl_tune_info), offsetof(dcdl_csc_info, beta_drift));
  printf("%zu %zu %d\\n", offsetof(dcdl_csc_opts, strategy), offsetof(dcdl_csc_opts, seed), (int)DCDL_SELECT_RANDOM);
  printf("%zu %zu %zu %zu\\n", offsetof(dcdl_csc_opts, refresh_limit), offsetof(dcdl_csc_info, t_init_corr_s),
         offsetof(dcdl_csc_info, n_corr64), offsetof(dcdl_csc_info, n_changed));
  printf("%zu %zu\\n", offsetof(dcdl_csc_opts, audit), offsetof(dcdl_csc_opts, audit_rounds));
  printf("%zu %zu %d\\n", offsetof(dcdl_csc_opts, fp64_method), offsetof(dcdl_csc_info, n_fft64),
         (int)DCDL_CORR_F64_FFT);
  return 0;
}
""")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(v) for v in lines[0].split()]
    offs = [int(v) for v in lines[1].split()]
    assert sizes == [ctypes.sizeof(dl.Shape), ctypes.sizeof(dl.CscOpts), ctypes.sizeof(dl.CscInfo)]
    assert offs == [dl.CscOpts.max_rounds.offset, dl.CscOpts.kkt_target.offset,
                    dl.CscInfo.converged.offset, dl.CscInfo.n_passes.offset]
    more = [int(v) for v in lines[2].split()]
    assert more == [ctypes.sizeof(dl.BatchOpts), ctypes.sizeof(dl.BatchInfo), ctypes.sizeof(dl.CscInfo),
                    dl.CscInfo.t_worker_apply_s.offset]
    srv = [int(v) for v in lines[3].split()]
    assert srv == [ctypes.sizeof(dl.ServerOpts), ctypes.sizeof(dl.ServerStats), dl.ServerOpts.tile.offset,
                   dl.ServerStats.t_busy_s.offset]
    dct = [int(v) for v in lines[4].split()]
    assert dct == [ctypes.sizeof(dl.DictOpts), ctypes.sizeof(dl.DictInfo), ctypes.sizeof(dl.CdlOpts),
                   ctypes.sizeof(dl.CdlInfo), dl.CdlOpts.dict.offset, dl.CdlInfo.n_updates.offset]
    last = [int(v) for v in lines[5].split()]
    assert last == [ctypes.sizeof(dl.TuneInfo), dl.CscInfo.beta_drift.offset]
    sel = [int(v) for v in lines[6].split()]
    assert sel == [dl.CscOpts.strategy.offset, dl.CscOpts.seed.offset, dl.SELECT["random"]]
    tail = [int(v) for v in lines[7].split()]
    assert tail == [dl.CscOpts.refresh_limit.offset, dl.CscInfo.t_init_corr_s.offset, dl.CscInfo.n_corr64.offset,
                    dl.CscInfo.n_changed.offset]
    aud = [int(v) for v in lines[8].split()]
    assert aud == [dl.CscOpts.audit.offset, dl.CscOpts.audit_rounds.offset]
    fft = [int(v) for v in lines[9].split()]
    assert fft == [dl.CscOpts.fp64_method.offset, dl.CscInfo.n_fft64.offset, dl.CORR_PREC["f64_fft"]]


def test_argument_checks_before_device_access(lib):
    import paper_1901_09235_amd as dl
    assert lib.dicodile_version().startswith(b"dicodile-mi355x")
    # NULL shape
    rc = lib.dicodile_dtd(None, 0, None, None, None)
    assert rc == -1 and b"shape" in lib.dicodile_last_error()
    s = dl.Shape()
    s.ndim, s.P, s.K = 3, 1, 1
    assert lib.dicodile_dtd(ctypes.byref(s), 0, None, None, None) == -1
    s.ndim, s.T[0], s.L[0] = 1, 10, 20  # L > T
    assert lib.dicodile_dtd(ctypes.byref(s), 0, ctypes.c_void_p(1), ctypes.c_void_p(1), None) == -1
    s.L[0] = 4
    o = dl.make_opts(-1.0, 0.0, 0)
    info = dl.CscInfo()
    rc = lib.dicodile_csc(ctypes.byref(s), ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.byref(o),
                          ctypes.c_void_p(1), ctypes.byref(info), None)
    assert rc == -1 and b"lambda" in lib.dicodile_last_error()
    o = dl.make_opts(1.0, 0.0, 0, strategy=4)
    rc = lib.dicodile_csc(ctypes.byref(s), ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.byref(o),
                          ctypes.c_void_p(1), ctypes.byref(info), None)
    assert rc == -1 and b"selection rule" in lib.dicodile_last_error()
    with pytest.raises(dl.DicodileError):
        dl.make_opts(1.0, 0.0, 0, strategy="sideways")
    # an apply table of K (2L1-1)(2L2-1) K entries beyond 32-bit offsets is
    # refused by the shape check, before any launch (K = 1024 atoms of 32x32)
    big = dl.Shape()
    big.ndim, big.P, big.K = 2, 1, 1024
    big.T[0], big.T[1], big.L[0], big.L[1] = 256, 256, 32, 32
    o = dl.make_opts(1.0, 0.0, 0)
    rc = lib.dicodile_csc(ctypes.byref(big), ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.byref(o),
                          ctypes.c_void_p(1), ctypes.byref(info), None)
    assert rc == -1 and b"32-bit offsets" in lib.dicodile_last_error()
    assert lib.dicodile_dtd(ctypes.byref(big), 0, ctypes.c_void_p(1), ctypes.c_void_p(1), None) == -1
    big.K = 256  # 256 * 63 * 63 * 256 = 2.6e8 entries: accepted by the shape check
    rc = lib.dicodile_csc(ctypes.byref(big), ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.byref(dl.make_opts(-1.0, 0.0, 0)),
                          ctypes.c_void_p(1), ctypes.byref(info), None)
    assert rc == -1 and b"lambda" in lib.dicodile_last_error()
    # the no-allocation solve refuses a problem beyond its fixed scratch before any device access
    s2 = dl.Shape()
    s2.ndim, s2.P, s2.K = 2, 1, 25
    s2.T[0], s2.T[1], s2.L[0], s2.L[1] = 1024, 1024, 16, 16
    rc = lib.dicodile_csc_noalloc(ctypes.byref(s2), ctypes.c_void_p(1), ctypes.c_void_p(1),
                                  ctypes.byref(dl.make_opts(1.0, 0.0, 0)), ctypes.c_void_p(1), ctypes.byref(info), None)
    assert rc == -1 and b"fixed scratch" in lib.dicodile_last_error()
    # server calls: NULL handles and arguments are rejected before any device access
    assert lib.dicodile_server_create(None, 0, None, None, None) == -1
    assert lib.dicodile_server_submit(None, None, None, None, None, None) == -1
    assert lib.dicodile_server_poll(None, 1, None) == -1
    assert lib.dicodile_server_wait(None, 1, 0.0, None) == -1
    assert lib.dicodile_server_stats(None, None) == -1
    assert lib.dicodile_server_destroy(None) == 0
    assert lib.dicodile_dict_update(None, 0, None, None, 0.0, None, None, None, None) == -1
    assert lib.dicodile_cdl(None, 0, None, None, None, None, None, None) == -1
    assert lib.dicodile_corr(None, 0, None, None, None, 0, None) == -1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_1901_09235_amd as dl
    monkeypatch.setattr(dl, "_lib", None)
    monkeypatch.setattr(dl, "_LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(dl.DicodileError):
        dl.load()


def test_oracle_builds_with_gcc():
    import oracle
    path = oracle.build(force=True)
    assert os.path.exists(path)
