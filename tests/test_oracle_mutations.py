"""Plant plausible mistakes in a copy of the oracle and check that a pin fails.

Each mutation edits one line of oracle.c in a temporary copy, rebuilds it
with gcc and runs the pin suite against the copy.  A mutation that every pin
lets through would show a hole in the pinning of the oracle.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = {
    "drop_one_body_creation": ("        Fp[c[j]] += f;", "        if (b[j] >= 0) Fp[c[j]] += f;"),
    "wrong_partner_index_a": ("            kd[a[j]] += k[j] * Y[b[j]];",
                              "            kd[a[j]] += k[j] * Y[a[j]];"),
    "wrong_partner_index_b": ("            kd[b[j]] += k[j] * Y[a[j]];",
                              "            kd[b[j]] += k[j] * Y[b[j]];"),
    "one_body_rate_times_Y": ("            kd[a[j]] += k[j];\n", "            kd[a[j]] += k[j] * Y[a[j]];\n"),
    "kappa_tie_to_euler": ("        if (kh < kappa) {", "        if (kh <= kappa) {"),
    "euler_sign": ("Yn[i] = Y[i] + h * (Fp[i] - kd[i] * Y[i]);",
                   "Yn[i] = Y[i] + h * (Fp[i] + kd[i] * Y[i]);"),
    "asymptotic_denominator": ("Yn[i] = (Y[i] + h * Fp[i]) / (1.0 + kh);",
                               "Yn[i] = (Y[i] + h * Fp[i]) / (1.0 + kd[i]);"),
    "growth_cap_ignored": ("fmin(o->grow_max, o->safety * o->tol / r)",
                           "fmax(o->grow_max, o->safety * o->tol / r)"),
    "clipped_step_sets_dt": ("            if (!clipped) {", "            if (1) {"),
    "shrink_floor_ignored": ("fmax(o->shrink_min, o->safety * o->tol / r)",
                             "fmin(o->shrink_min, o->safety * o->tol / r)"),
    "change_against_new_state": ("fabs(Yn[i] - Y[i]) / fmax(Y[i], y_floor)",
                                 "fabs(Yn[i] - Y[i]) / fmax(Yn[i], y_floor)"),
    "accept_threshold": ("int accept = r <= o->tol;", "int accept = r < 0.5 * o->tol;"),
    # single precision
    "f32_euler_sign": ("yf[i] + hf * (fpf[i] - kdf[i] * yf[i])", "yf[i] + hf * (fpf[i] + kdf[i] * yf[i])"),
    "f32_asymptotic_denominator": ("/ (1.0f + khf)", "/ (1.0f + kdf[i])"),
    "f32_partner_index": ("kdf[ra[j]] += kj * yf[rb[j]];", "kdf[ra[j]] += kj * yf[ra[j]];"),
    "f32_change_against_new_state": ("fmaxf(yf[i], floorf_)", "fmaxf(ynf[i], floorf_)"),
    "f32_state_kept_double": ("        Yf[i] = (float)Y[i];", "        Yf[i] = (float)(Y[i] * 1.0000001);"),
    # chunked sums of long rows
    "chunk_not_multiple_of_4": ("    const int32_t chunk = split_above / 2 / 4 * 4;",
                                "    const int32_t chunk = split_above / 2;"),
    "row_of_split_above_terms_split": ("    if (split_above <= 0 || n <= split_above) {\n        double s",
                                       "    if (split_above <= 0 || n < split_above) {\n        double s"),
    "chunk_sum_not_restarted": ("        double s = 0.0;\n        for (int32_t q = first;",
                                "        double s = total;\n        for (int32_t q = first;"),
    "f32_chunk_sum_not_restarted": ("        float s = 0.0f;\n        for (int32_t q = first;",
                                    "        float s = total;\n        for (int32_t q = first;"),
}

# mistakes in the learned-controller reference (the part of oracle.c after LEARNED_MARK)
LEARNED_MUTATIONS = {
    "learned_no_plain_fallback": ("                step = plain_step;", "                step = h * 0.5;"),
    "learned_mean_feature_unscaled": ("fmax(ksum / n_species, 1e-300)", "fmax(ksum, 1e-300)"),
    "learned_label_no_safety": ("log2(o->safety) + lo / 32.0", "lo / 32.0"),
    "learned_label_against_new_state": ("orc_change(n_species, Y, Yn, o->y_floor) <= o->tol",
                                        "orc_change(n_species, Yn, Y, o->y_floor) <= o->tol"),
    "learned_bias_dropped": ("        a += b2[j];\n", "\n"),
    "learned_relu_before_bias": ("        a += b1[j];\n        h1[j] = orc_bf16(a > 0.0 ? a : 0.0);",
                                 "        h1[j] = orc_bf16(a > 0.0 ? a : 0.0) + b1[j];"),
    "learned_q_floor": ("q32 = (int32_t)rint(32.0 * fmin(fmax(ov, -3.0), 3.0));",
                        "q32 = (int32_t)floor(32.0 * fmin(fmax(ov, -3.0), 3.0));"),
}
LEARNED_MARK = "Learned step proposer"


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS) + sorted(LEARNED_MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    learned = name in LEARNED_MUTATIONS
    before, after = (LEARNED_MUTATIONS if learned else MUTATIONS)[name]
    dst = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), dst,
                    ignore=shutil.ignore_patterns("*.so", "*.tmp", "__pycache__"))
    src = (dst / "oracle.c").read_text()
    cut = src.index(LEARNED_MARK)
    head, tail = src[:cut], src[cut:]
    if learned:
        assert tail.count(before) == 1, "mutation site not found: the oracle changed"
        tail = tail.replace(before, after)
    else:
        assert head.count(before) == 1, "mutation site not found: the oracle changed"
        head = head.replace(before, after)
    (dst / "oracle.c").write_text(head + tail)
    env = dict(os.environ, PYTHONPATH=f"{tmp_path}{os.pathsep}{ROOT}")
    # every pin file runs; the one a mutation of its kind most likely fails goes first (-x)
    files = ["test_oracle_pins.py", "test_mlp_oracle.py", "test_oracle_f32.py"]
    first = ("test_oracle_f32.py" if name.startswith("f32_") else
             "test_mlp_oracle.py" if learned else "test_oracle_pins.py")
    files.remove(first)
    files.insert(0, first)
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                          *[os.path.join(ROOT, "tests", f) for f in files]],
                         env=env, cwd=str(tmp_path), capture_output=True, text=True, timeout=300)
    assert res.returncode != 0, f"no pin failed for mutation {name}:\n{res.stdout[-2000:]}"
    # and the copy really was the one under test
    assert (dst / "liboracle.so").exists()
