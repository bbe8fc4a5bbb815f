"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a COPY of oracle/oracle.c (on the CPU, in a
temporary directory), builds it, and runs a selection of the pin tests
against that build in a child process: the selection must fail.  A control
build of the unmodified source must pass the same selection, so a failure
means the planted mistake was caught, not that the harness broke.

The mistakes are the ones a reader of Sec. 5.2-5.3 could plausibly make:
the shifted-ReLU derivative tested at s > 0 instead of s + 1/2 > 0, a
backward that ignores early termination or the sample cap its forward
applied, an exclusive instead of inclusive prefix in Eq. 9/10, T_i instead
of T_{i+1}, the position chain of Eq. 14 without the t_i factor, and the
sign of the L1 depth derivative; and, for records of SH degree 0 and 1, a
channel offset that keeps the degree-2 stride of nine, a record stride that
ignores the padding of degree-1 records, and a gradient scattered with the
degree-2 record stride.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PINS = ["tests/test_oracle_pins_workload_settings.py", "tests/test_oracle_pins.py",
        "tests/test_oracle_pins_sh_degree.py"]

MUTATIONS = {
    "relu_shift_derivative_at_s_gt_0": (
        "return s + 0.5 > 0.0 ? 1.0 : 0.0;",
        "return s > 0.0 ? 1.0 : 0.0;",
        "shifted_relu"),
    "backward_ignores_early_termination": (
        "    march(g, op, o, d, tr);\n    /* the loss sees",
        "    oopts op2 = *op; op2.t_stop = 0.0; march(g, &op2, o, d, tr);\n    /* the loss sees",
        "early_termination"),
    "backward_ignores_the_cap": (
        "    march(g, op, o, d, tr);\n    /* the loss sees",
        "    oopts op2 = *op; op2.max_samples = 1 << 30; march(g, &op2, o, d, tr);\n    /* the loss sees",
        "binding_sample_cap"),
    "exclusive_prefix_in_eq9": (
        "(tr->c[i][ch] * Tn - tr->rgb[ch] + prefC[ch])",
        "(tr->c[i][ch] * Tn - tr->rgb[ch] + prefC[ch] - tr->c[i][ch] * tr->w[i])",
        "shifted_relu or grid_backward_matches"),
    "T_i_instead_of_T_i_plus_1": (
        "const double Tn = tr->T[i + 1];",
        "const double Tn = tr->T[i];",
        "shifted_relu or grid_backward_matches"),
    "pose_direction_chain_without_t": (
        "gd[a] += tr->t[i] * gp[a];",
        "gd[a] += gp[a];",
        "pose_backward"),
    "l1_depth_sign_flipped": (
        "drho = e > 0.0 ? 1.0 : (e < 0.0 ? -1.0 : 0.0);",
        "drho = e > 0.0 ? -1.0 : (e < 0.0 ? 1.0 : 0.0);",
        "loss_gradient_fd"),
    "reduced_degree_channel_offset_of_nine": (
        "for (int kk = 0; kk < g->nsh; ++kk) acc += Y[kk] * val[1 + ch * g->nsh + kk];",
        "for (int kk = 0; kk < g->nsh; ++kk) acc += Y[kk] * val[1 + ch * NSH + kk];",
        "degree0 or degree1 or reduced_degree"),
    "degree1_record_without_padding": (
        "g->stride = deg == 0 ? 4 : deg == 1 ? 16 : NREC;",
        "g->stride = deg == 0 ? 4 : deg == 1 ? 13 : NREC;",
        "degree1 or reduced_degree"),
    "reduced_degree_gradient_with_degree2_stride": (
        "double *dst = grad_data + cc.idx[b] * g->stride;",
        "double *dst = grad_data + cc.idx[b] * (g->stride < NREC ? g->nrec : g->stride);",
        "degree1_grid_backward or reduced_degree"),
}


def _run_pins(lib_path, selection):
    env = dict(os.environ, PXM_ORACLE_LIB=lib_path)
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *PINS,
           "-k", selection]
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)


@pytest.fixture(scope="module")
def source():
    with open(SRC) as fh:
        return fh.read()


def test_control_build_passes_every_selection(source, tmp_path):
    lib = oracle.build(src=SRC, out=str(tmp_path / "control.so"))
    sels = sorted({sel for _, _, sel in MUTATIONS.values()})
    res = _run_pins(lib, " or ".join(f"({s})" for s in sels))
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-2000:]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(source, tmp_path, name):
    old, new, sel = MUTATIONS[name]
    assert source.count(old) == 1, f"mutation site of {name} not unique in oracle.c"
    src = tmp_path / f"{name}.c"
    src.write_text(source.replace(old, new))
    lib = oracle.build(src=str(src), out=str(tmp_path / f"{name}.so"))
    res = _run_pins(lib, sel)
    assert res.returncode == 1, f"{name} was not caught:\n" + res.stdout[-2000:]
