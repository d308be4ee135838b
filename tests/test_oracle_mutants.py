"""Each plausible mistake planted in the oracle (on the CPU, in a private copy
of its source) must make at least one of the oracle's pin tests fail."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "tpx_oracle.c")
PINS = ["tests/test_oracle_paper_example.py", "tests/test_oracle_vs_bruteforce.py",
        "tests/test_oracle_invariants.py", "tests/test_oracle_decode.py",
        "tests/test_oracle_paper_mode.py"]

MUTANTS = {
    "spatial_off_by_one": ("orc_absdiff(x[i], x[j]) <= dxy", "orc_absdiff(x[i], x[j]) < dxy"),
    "time_window_exclusive": ("toa[j] - toa[i] > dt_ticks) break;", "toa[j] - toa[i] >= dt_ticks) break;"),
    "root_is_max": ("if (ra < rb) parent[rb] = ra; else parent[ra] = rb;",
                    "if (ra > rb) parent[rb] = ra; else parent[ra] = rb;"),
    "x_moment_uses_y": ("Sx[r] += (int64_t)tot[i] * x[i];", "Sx[r] += (int64_t)tot[i] * y[i];"),
    "y_weight_dropped": ("Sy[r] += (int64_t)tot[i] * y[i];", "Sy[r] += (int64_t)y[i];"),
    "wrap_sign": ("u->epoch += 1;", "u->epoch -= 2;"),
    "late_reporter_ignored": ("u->epoch -= 1;", "u->epoch -= 0;"),
    "assign_lower_bound": ("if (trig[mid] <= ti) lo = mid + 1;", "if (trig[mid] < ti) lo = mid + 1;"),
    "tof_cut_exclusive": ("if (tof > p->tof_max_ticks)", "if (tof >= p->tof_max_ticks)"),
    "decode_x_bit": ("*x = 2 * dcol + (pix >> 2);", "*x = 2 * dcol + (pix & 1);"),
    "decode_y_bits": ("*y = 4 * spix + (pix & 3);", "*y = 4 * spix + (pix >> 1);"),
    "fine_toa_sign": ("*raw = ((coarse << 4) - ftoa)", "*raw = ((coarse << 4) + ftoa)"),
    "tdc_stamp_shift": ("uint64_t stamp = (w >> 9)", "uint64_t stamp = (w >> 8)"),
    "shots_merge": ("if (shot[j] != shot[i] || toa[j] - toa[i] > dt_ticks) break;",
                    "if (toa[j] - toa[i] > dt_ticks) break;"),
    "walk_sign": ("(ORC_TICK_NS * (double)St[r] - Sw[r])", "(ORC_TICK_NS * (double)St[r] + Sw[r])"),
    "tof_from_first_trigger": ("int64_t tof = (int64_t)(toa[i] - trig[shot[i]]);",
                               "int64_t tof = (int64_t)(toa[i] - trig[0]);"),
    "toa_first_max": ("if (toa[i] < tmin[r]) tmin[r] = toa[i];",
                      "if (toa[i] > tmin[r] || tmin[r] == UINT64_MAX) tmin[r] = toa[i];"),
    "unweighted_mean_denominator": ("h->x = (double)Ux[r] / (double)cnt[r];",
                                    "h->x = (double)Ux[r] / (double)(cnt[r] + 1);"),
    "hit_order_by_label_only": ("if (g_root_shot[i] != g_root_shot[j])", "if (0)"),
    "wrap_counter_not_counted": ("(*u->n_wraps)++;", ";"),
    # paper mode (local maxima, Eq. 9 on A)
    "paper_tie_break_reversed": ("(tot[j] == tot[i] && j > i)", "(tot[j] == tot[i] && j < i)"),
    "paper_ties_all_maxima": ("if (tot[j] > tot[i] || (tot[j] == tot[i] && j > i)) is_max = 0;",
                              "if (tot[j] > tot[i]) is_max = 0;"),
    "paper_row_without_self": ("if (j != i && !orc_nb(x, y, toa, i, j, dxy, dt_ticks)) continue;",
                               "if (j == i || !orc_nb(x, y, toa, i, j, dxy, dt_ticks)) continue;"),
    "paper_time_ignored": (" && (d < 0 ? -d : d) <= dt;", ";"),
    "paper_row_unweighted": ("Sx += (int64_t)tot[j] * x[j];", "Sx += x[j];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    anchor, repl = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(anchor) == 1, f"anchor for {name} not found exactly once"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "mut.c")
        so = os.path.join(d, "libmut.so")
        open(c, "w").write(src.replace(anchor, repl))
        subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", c, "-o", so])
        env = dict(os.environ, TPX_ORACLE_LIB=so)
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            "--hypothesis-seed=0", *PINS], cwd=ROOT, env=env,
                           capture_output=True, text=True, timeout=300)
        assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-800:]}"
