"""Planted mistakes in the oracle must each fail at least one pin.

Each case below copies oracle/ffs_oracle.c, plants one plausible mistake (a
dropped term, a flipped comparison, a wrong index, direction, boundary or
constant), builds the copy on the CPU and runs the oracle's pin tests against
it (FFS_ORACLE_LIB points the oracle package at the copy). A case passes when
the pins fail. This checks the pins, not the oracle: a mistake that no pin
notices would also go unnoticed in the GPU parity tests, which are held to the
oracle.
"""
import concurrent.futures
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ffs_oracle.c")
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_init_work.py", "tests/test_oracle_xy.py",
        "tests/test_oracle_rules.py", "tests/test_oracle_static.py",
        "tests/test_oracle_schemes.py"]

# (name, text in ffs_oracle.c (must occur once), replacement)
MUTANTS = [
    # decoder: power limit, push-right window, placement, machine choice
    ("power limit not strict", "if (d->profile[tau - in->rs] + q > in->q_max) last_bad = tau;",
     "if (d->profile[tau - in->rs] + q >= in->q_max) last_bad = tau;"),
    ("window one slot short when committed",
     "for (int64_t tau = t; tau < (int64_t)t + p; ++tau) d->profile[tau - in->rs] += q;",
     "for (int64_t tau = t; tau < (int64_t)t + p - 1; ++tau) d->profile[tau - in->rs] += q;"),
    ("running ops hold power one slot short",
     "for (int64_t tau = 0; tau < (int64_t)end - in->rs; ++tau) d->profile[tau] += q;",
     "for (int64_t tau = 0; tau < (int64_t)end - in->rs - 1; ++tau) d->profile[tau] += q;"),
    ("earliest start ignores RS", "const int32_t est = MAX32(in->rs, d->done_at[j]);",
     "const int32_t est = d->done_at[j];"),
    ("machine not append-only", "const int32_t t0 = MAX32(est, free_s[m]);",
     "const int32_t t0 = est;"),
    ("machine choice ignores machine free time",
     "int32_t end = MAX32(est, free_s[c]) + P_AT(in, j, s, c);",
     "int32_t end = est + P_AT(in, j, s, c);"),
    ("machine choice ties to the highest index", "if (m < 0 || end < best_end) {",
     "if (m < 0 || end <= best_end) {"),
    ("priority order reversed", "order[n - pk] = in->active[k];", "order[pk - 1] = in->active[k];"),
    # objective, eqs. (1)-(3)
    ("tardiness sign", "int32_t late = c - in->due[j];", "int32_t late = in->due[j] - c;"),
    ("tardiness weight dropped", "return (int64_t)in->wt * tardiness + cmax;",
     "return tardiness + cmax;"),
    ("frozen makespan dropped", "int32_t cmax = in->frozen_cmax;", "int32_t cmax = 0;"),
    # work count
    ("work: updated slots dropped",
     "d->work += machine == -2 ? (int64_t)p : (int64_t)(t - t0) + 2 * (int64_t)p;",
     "d->work += machine == -2 ? (int64_t)p : (int64_t)(t - t0) + (int64_t)p;"),
    ("work: machine comparisons miscounted",
     "d->work += 3;\n      if (m < 0 || end < best_end)", "d->work += 2;\n      if (m < 0 || end < best_end)"),
    # rescheduling (Section 4.1, eq. (10), Algorithm 1)
    ("op starting at RS frozen", "if (plan_start[(int64_t)j * g + s] >= rs) {",
     "if (plan_start[(int64_t)j * g + s] > rs) {"),
    ("op ending at RS counted as running", "if (end > rs) {  /* running",
     "if (end >= rs) {  /* running"),
    ("resumed job ready at its release", "out->ready[j] = f == 0 ? prev->release[j] : last_end;",
     "out->ready[j] = prev->release[j];"),
    ("frozen machine free time dropped",
     "if (end > out->machine_free[s * om + m]) out->machine_free[s * om + m] = end;", ";"),
    # the traditional static approach (Fig. 7)
    ("static: arrivals after each machine's last op, not the stage's",
     "out->machine_free[s * om + m] = m < prev->n_machines[s] ? stage_end[s] : 0;",
     "out->machine_free[s * om + m] = 0;"),
    ("static: unstarted planned ops hold no power",
     "      d->profile[tau] += q;\n  }\n  return ORC_OK;", "      ;\n  }\n  return ORC_OK;"),
    ("static: op running at RS dropped", "if (st < rs && end > rs) {  /* running at RS",
     "if (0) {  /* running at RS"),
    # the comparison GAs of Section 5.2
    ("E_max one power of ten short", "if (below || e > INT64_MAX / 10) return e;",
     "if (below || e > INT64_MAX / 10) return e / 10 > 1 ? e / 10 : e;"),
    ("roulette picks the first sum at or above the target", "if (prefix[i] > hi) return i;",
     "if (prefix[i] >= hi) return i;"),
    ("roulette fitness without the zero floor", "total += f > 0 ? (uint64_t)f : 0;",
     "total += (uint64_t)f;"),
    ("cellular second parent is the worst", "if (k != b1 && (b2 < 0 || obj_in[cand[k]] < obj_in[cand[b2]])) b2 = k;",
     "if (k != b1 && (b2 < 0 || obj_in[cand[k]] > obj_in[cand[b2]])) b2 = k;"),
    ("cellular replaces on ties", "const int better = cobj[i] < obj_in[i];",
     "const int better = cobj[i] <= obj_in[i];"),
    ("cellular always replaces", "const int better = cobj[i] < obj_in[i];", "const int better = 1;"),
    # random numbers and initialisation
    ("Philox key schedule", "k0 += W0;", "k0 += W1;"),
    ("Sattolo shuffle", "int32_t r = (int32_t)draw_below(w[d % 4], (uint32_t)(pos + 1));",
     "int32_t r = (int32_t)draw_below(w[d % 4], (uint32_t)(pos));"),
    ("shuffle word order", "int32_t r = (int32_t)draw_below(w[d % 4], (uint32_t)(pos + 1));",
     "int32_t r = (int32_t)draw_below(w[3 - d % 4], (uint32_t)(pos + 1));"),
    ("initial elite is the worst", "if (obj[i] < obj[b]) b = i;", "if (obj[i] > obj[b]) b = i;"),
    # GA operators (Section 4.4)
    ("selection ties to the last", "if (obj[cand[k]] < obj[w]) w = cand[k];",
     "if (obj[cand[k]] <= obj[w]) w = cand[k];"),
    ("selection neighbour off the torus", "base + ((r + 1) % R) * C + c,",
     "base + ((r + 2) % R) * C + c,"),
    ("crossover pairing parity", "const int horizontal = gen % 2 == 1;",
     "const int horizontal = gen % 2 == 0;"),
    ("crossover cut may be 0",
     "int32_t cut = 1 + (int32_t)draw_below(w[1], (uint32_t)(n_genes - 1));",
     "int32_t cut = (int32_t)draw_below(w[1], (uint32_t)(n_genes - 1));"),
    ("crossover head one gene long",
     "child_a[k] = k < cut ? a[k] : b[k];\n    child_b[k] = k < cut ? b[k] : a[k];\n  }\n  orc_correct(n, child_a);",
     "child_a[k] = k <= cut ? a[k] : b[k];\n    child_b[k] = k <= cut ? b[k] : a[k];\n  }\n  orc_correct(n, child_a);"),
    ("correction fills the largest missing first", "v[k] = missing;\n    seen[missing] = 1;",
     "v[k] = n + 1 - missing;\n    seen[missing] = 1;"),
    ("mutation may swap a gene with itself", "if (y >= x) ++y;", "if (y > x) ++y;"),
    ("mutation probability inverted", "if ((uint32_t)(w[0] >> 32) >= gp->pm) continue;",
     "if ((uint32_t)(w[0] >> 32) < gp->pm) continue;"),
    ("replacement keeps a worse elite", "if (obj_out[b] < elite_obj_out[I]) {",
     "if (obj_out[b] > elite_obj_out[I]) {"),
    ("replacement worst ties to the last", "if (obj_out[i] > obj_out[w]) w = i;",
     "if (obj_out[i] >= obj_out[w]) w = i;"),
    ("migration ring direction", "const int32_t src = (I - 1 + I_n) % I_n;",
     "const int32_t src = (I + 1) % I_n;"),
    ("migration overwrites the best",
     "if (!taken[i] && (w < 0 || obj_out[I * K + i] > obj_out[I * K + w])) w = i;",
     "if (!taken[i] && (w < 0 || obj_out[I * K + i] < obj_out[I * K + w])) w = i;"),
]


def _build_and_run(name, old, new, tmp):
    src = open(SRC).read()
    assert src.count(old) == 1, f"{name}: text to mutate must occur exactly once"
    tag = "".join(c if c.isalnum() else "_" for c in name)
    cfile = os.path.join(tmp, f"{tag}.c")
    lib = os.path.join(tmp, f"{tag}.so")
    with open(cfile, "w") as f:
        f.write(src.replace(old, new))
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-w", "-I",
                    os.path.dirname(SRC), "-o", lib, cfile],
                   check=True)
    env = dict(os.environ, FFS_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=240)
        return name, r.returncode, r.stdout[-400:]
    except subprocess.TimeoutExpired:
        return name, "timeout", ""


def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            results = list(ex.map(lambda m: _build_and_run(*m, tmp), MUTANTS))
    survivors = [(name, out) for name, rc, out in results if rc == 0]
    assert not survivors, "planted mistakes no pin catches:\n" + "\n".join(
        f"{n}: {o}" for n, o in survivors)
    # pytest's exit status 1 = some test failed; anything else is a broken run
    broken = [(n, rc) for n, rc, _ in results if rc not in (1, "timeout")]
    assert not broken, broken


def test_unmutated_copy_passes_the_pins():
    """The harness itself: the oracle's own source built the same way passes."""
    with tempfile.TemporaryDirectory() as tmp:
        name, rc, out = _build_and_run("unmutated", "k0 += W0;", "k0 += W0;", tmp)
    assert rc == 0, out
