"""Host-side checks of the C-ABI library: it loads, exports every function the
header declares, its structs match the ctypes mirrors, and the host-only calls
work.  No GPU call is made here."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rlobpcg.h")


def _lib_or_skip():
    import paper_2602_16797_amd as rl
    if not os.path.exists(rl.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    return rl, rl.load_library()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rl_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("rl_create", "rl_destroy", "rl_default_opts", "rl_svds_smallest_d", "rl_svds_smallest_z",
                 "rl_step_sketch", "rl_step_qr", "rl_step_astream", "rl_step_astream_iter", "rl_step_tall_svd", "rl_step_orth", "rl_status_string",
                 "rl_step_sketch_f32", "rl_step_qr_lowp", "rl_server_create", "rl_server_submit",
                 "rl_server_poll", "rl_server_wait", "rl_server_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    rl, lib = _lib_or_skip()
    out = subprocess.run(["nm", "-D", "--defined-only", rl.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (rl_[a-z0-9_]+)\b", out))
    for name in _declared():
        assert name in exported, name
        assert hasattr(lib, name)
    assert set(rl.EXPORTED) <= exported


def test_struct_layout_matches_ctypes(tmp_path):
    rl, _ = _lib_or_skip()
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "rlobpcg.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(rl_opts), sizeof(rl_info),"
        " offsetof(rl_opts, tau), offsetof(rl_opts, lanczos_steps), offsetof(rl_info, sigma1),"
        " offsetof(rl_info, hist_cap), offsetof(rl_info, rnorm_hist));"
        "printf(\"%zu %zu %zu %zu %zu\\n\", offsetof(rl_info, n_pass_g), offsetof(rl_info, t_pass_g_us),"
        " offsetof(rl_opts, refresh), offsetof(rl_opts, prec_guard), offsetof(rl_info, kappa_est));"
        "printf(\"%zu %zu %zu\\n\", offsetof(rl_opts, sketch_prec), offsetof(rl_opts, loop_precond), offsetof(rl_opts, orth));"
        "printf(\"%zu %zu %zu\\n\", offsetof(rl_opts, lock), offsetof(rl_info, n_locked), offsetof(rl_info, act_mask));"
        "printf(\"%zu %zu %zu %zu\\n\", sizeof(rl_request), offsetof(rl_request, opts), offsetof(rl_request, ldu),"
        " sizeof(rl_job_times));return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    O, I = rl.RlOpts, rl.RlInfo
    assert vals == [ctypes.sizeof(O), ctypes.sizeof(I), O.tau.offset, O.lanczos_steps.offset, I.sigma1.offset,
                    I.hist_cap.offset, I.rnorm_hist.offset, I.n_pass_g.offset, I.t_pass_g_us.offset, O.refresh.offset,
                    O.prec_guard.offset, I.kappa_est.offset,
                    O.sketch_prec.offset, O.loop_precond.offset, O.orth.offset,
                    O.lock.offset, I.n_locked.offset, I.act_mask.offset,
                    ctypes.sizeof(rl.RlRequest), rl.RlRequest.opts.offset, rl.RlRequest.ldu.offset,
                    ctypes.sizeof(rl.RlJobTimes)]


def test_host_only_calls():
    rl, lib = _lib_or_skip()
    o = rl.default_opts(10_000, 200, 1)
    assert o.d == 800 and o.zeta == 8 and o.block == 1 and o.max_iter == 200 and o.check_every == 5
    assert o.tau == 2.0 * 200 ** 0.5 * 2.0 ** -52
    assert o.sketch_prec == rl.RL_SKETCH_F64
    assert o.refresh == 1 and o.prec_guard == 1 and o.lock == 0
    assert rl.default_opts(10_000, 200, 3).max_iter == 100
    # wide real shapes default to the plain-sum pass (the only one past n = 1024)
    assert rl.default_opts(10_000, 1024, 1).dot2 == 1
    assert rl.default_opts(100_000, 2000, 1).dot2 == 0
    assert rl.status_string(rl.RL_ERR_ARG) == "invalid argument"
    assert lib.rl_default_opts(None, 1, 1, 1) == rl.RL_ERR_ARG
    # argument errors are caught on the host before any device work
    assert lib.rl_svds_smallest_d(None, 10, 5, None, 5, 1, None, None, None, 1, None, 1, None) == rl.RL_ERR_ARG
    assert lib.rl_destroy(None) == rl.RL_OK
