"""Plausible mistakes planted in a copy of the oracle must fail some pin.

Each case edits one spot of oracle.c (a dropped term, a wrong sign or index,
swapped operands), builds the copy with gcc and runs all pins on it in a child
process.  This shows the pins would catch such a mistake in the oracle itself.
"""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "oracle.c")

PLANTS = {
    "network_comparator_reversed": (
        "        if (rec_less(o, y, x)) {\n            rec_t t = *x;",
        "        if (rec_less(o, x, y)) {\n            rec_t t = *x;"),
    "batcher_merge_skips_last_comparator": (
        "for (int i = lo + r; i + r < lo + n; i += step)",
        "for (int i = lo + r; i + r < lo + n - step; i += step)"),
    "redundant_comparators_kept": (
        "            if (useful[c]) {", "            if (1) {"),
    "merge_prefers_right_on_ties": (
        "            from_right = rec_less(&c->ord, &right[ri], &left[li]);",
        "            from_right = !rec_less(&c->ord, &left[li], &right[ri]);"),
    "merge_drops_left_tail": (
        "        else if (ri == nr)\n            from_right = 0;",
        "        else if (ri == nr)\n            break;"),
    "merge_split_off_by_one": (
        "            merge_neighbours(c, a, r.start, nl, r.count);",
        "            merge_neighbours(c, a, r.start, nl - (nl > 1), r.count);"),
    "quick_sort_skips_element": (
        "            const range_t hi = {cut + 1, last - cut, 0};",
        "            const range_t hi = {cut + 2, last - cut - 1, 0};"),
    "tie_break_reversed": (
        "    return o->stable && a->pos < b->pos;", "    return o->stable && a->pos > b->pos;"),
    "int32_compared_unsigned": (
        "    if (dtype == ORC_I32) return (int32_t)a < (int32_t)b;",
        "    if (dtype == ORC_I32) return a < b;"),
    "f32_compared_as_bits": (
        "        return fa < fb;                  /* IEEE: -0 < +0 is false       */",
        "        return a < b;"),
    "f32_nan_first": (
        "        if (isnan(fb)) return 1;", "        if (isnan(fb)) return 0;"),
    "table3_even_missing_6": (
        '{"Even", (1u << 4) | (1u << 6) | (1u << 8)}', '{"Even", (1u << 4) | (1u << 8)}'),
    "network_dispatch_off_by_one": (
        "            apply_network(&c->ord, a + r.start, (int)r.count);",
        "            apply_network(&c->ord, a + r.start, (int)r.count - 1);"),
    "backward_scatters_the_wrong_way": (
        "            grad_in[r * cols + perm[r * cols + i]] = grad_out[r * cols + i];",
        "            grad_in[r * cols + i] = grad_out[r * cols + perm[r * cols + i]];"),
}


def test_clean_oracle_passes_runner(tmp_path):
    so = oracle.build(SRC, str(tmp_path / "clean.so"))
    r = subprocess.run([sys.executable, os.path.join(HERE, "plant_runner.py"), so],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.parametrize("name", sorted(PLANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = PLANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"plant site for {name} not found exactly once"
    src = tmp_path / "planted.c"
    src.write_text(text.replace(old, new))
    so = oracle.build(str(src), str(tmp_path / "planted.so"))
    r = subprocess.run([sys.executable, os.path.join(HERE, "plant_runner.py"), so],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"{name} passed every pin:\n{r.stdout}{r.stderr}"


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    # every pin against the oracle built with AddressSanitizer and
    # UndefinedBehaviorSanitizer; any finding aborts the child process
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    so = oracle.build(SRC, str(tmp_path / "sanitized.so"),
                      extra=("-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                             "-fno-sanitize-recover=all"))
    env = dict(os.environ)
    env["LD_PRELOAD"] = " ".join(p for p in (asan, _runtime("libubsan.so")) if p)
    # Python's own allocations are not instrumented; leaks at exit are not the oracle's
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, os.path.join(HERE, "plant_runner.py"), so],
                       capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "failed: none" in r.stdout
