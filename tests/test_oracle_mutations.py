"""Planted mistakes: each mutation of the oracle's source (on a copy, compiled
on the CPU) must make the pin suite fail.  This shows the pins would catch a
dropped term, a wrong sign, a swapped index or a transposed operand."""
import os
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "qtm_oracle.c")

MUTATIONS = {
    "rx_offdiag_sign": ("u[0][1] = -I * s;", "u[0][1] = I * s;"),
    "ry_transposed": ("u[0][0] = c;  u[0][1] = -s;\n    u[1][0] = s;",
                      "u[0][0] = c;  u[0][1] = s;\n    u[1][0] = -s;"),
    "rz_phase_sign": ("u[0][0] = cexp(-I * t / 2);", "u[0][0] = cexp(I * t / 2);"),
    "cnot_ctl_tgt_swapped": ("apply_cnot(psi, n, g[1], g[2], par);", "apply_cnot(psi, n, g[2], g[1], par);"),
    "ry_deriv_dropped_half": ("d[1][0] = c / 2;", "d[1][0] = c;"),
    "reverse_not_daggered": ("apply_gate(phi, c->n, g, x_b, w, 1, par);", "apply_gate(phi, c->n, g, x_b, w, 0, par);"),
    "zsign_flipped": ("& 1) ? -1.0 : 1.0;", "& 1) ? 1.0 : -1.0;"),
    "bra_drops_G": ("dsum += J->G[(int64_t)b * M + m] * zsign(x, c->masks[m]);", "dsum += zsign(x, c->masks[m]);"),
    "cz_or_not_and": ("if ((x & ab) && (x & bb)) psi[x] = -psi[x];", "if ((x & ab) || (x & bb)) psi[x] = -psi[x];"),
    "last_gate_dropped": ("for (int k = 0; k < c->n_gates; ++k)\n    apply_gate", "for (int k = 0; k < c->n_gates - 1; ++k)\n    apply_gate"),
    "grad_x_wrong_slot": ("if (xrow) xrow[gk[4]] += v;\n",
                          "if (xrow) xrow[(gk[4] + 1) % c->n_inputs] += v;\n"),
    "scaled_angle_unscaled": ("if (g[3] == O_SRC_SCALED) return w[g[2]] * x_b[g[4]];",
                              "if (g[3] == O_SRC_SCALED) return x_b[g[4]];"),
    "scaled_grad_w_no_input_factor": ("wrow[gk[2]] += v * x_b[gk[4]];", "wrow[gk[2]] += v;"),
    "scaled_grad_x_no_weight_factor": ("if (xrow) xrow[gk[4]] += v * J->w[gk[2]];",
                                       "if (xrow) xrow[gk[4]] += v;"),
    "pauli_y_conjugated": ("u[0][0] = 0;  u[0][1] = -I;\n      u[1][0] = I;",
                           "u[0][0] = 0;  u[0][1] = I;\n      u[1][0] = -I;"),
    "pauli_x_taken_as_z": ("} else if (xb) {", "} else if (0) {"),
    "pauli_bra_drops_G": ("lam[j][x] += gm * mu[x];", "lam[j][x] += mu[x];"),
    "h_sign_on_wrong_entry": ("case 5:  u[0][0] = r; u[0][1] = r; u[1][0] = r; u[1][1] = -r;",
                              "case 5:  u[0][0] = r; u[0][1] = -r; u[1][0] = r; u[1][1] = r;"),
    "s_phase_conjugated": ("case 9:  u[1][1] = I;", "case 9:  u[1][1] = -I;"),
    "crot_control_ignored": ("if ((x & bit) || !(x & cb)) continue;", "if (x & bit) continue;"),
    "crot_derivative_unmasked": ("          if (!(x & cb)) mu[x] = 0;\n", "          (void)cb;\n"),
    "split_remainder_last": ("*lo = t * base + (t < rem ? t : rem);\n  *hi = *lo + base + (t < rem ? 1 : 0);",
                             "*lo = t * base + (t > T - 1 - rem ? t - (T - rem) : 0);\n  *hi = *lo + base + (t >= T - rem ? 1 : 0);"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found exactly once: {name}"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fcx-limited-range",
                    "-o", str(lib), str(mut), "-lm"], check=True)
    env = dict(os.environ, QTM_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"planted mistake {name} was not caught:\n{r.stdout[-2000:]}"
