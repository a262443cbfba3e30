"""The oracle's pins catch plausible mistakes.

Each mutation below is a mistake someone could make while writing the
oracle: a wrong element mapping, a missing or extra rounding, a wrong
padding value, a reordered compensation, an off-by-one in a shuffle or
scan bound, a wrong predicate or mask, a flipped comparator, an unstable
insertion, an inverted step size, a misplaced output.  It is applied to a scratch copy of coxo.c, built on the CPU
with the oracle's own flags, and the oracle's pin suites run against that
build in a subprocess: at least one pin must fail.  (The committed oracle
passes them all, in the rest of the test suite.)
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "coxo.c")
PINS = ["tests/test_oracle_kernels.py", "tests/test_oracle_semantics.py", "tests/test_oracle_image.py",
        "tests/test_oracle_cg.py"]

MUTATIONS = [
    ("bf16 rows of 4 elements instead of 8",
     "  int v = dtype == DT_BF16 ? 8 : 4;", "  int v = dtype == DT_BF16 ? 4 : 4;"),
    ("plain dot as a rounded product plus s instead of one fmaf",
     "      a->s = fmaf(xv, yv, a->s);", "      a->s = xv * yv + a->s;"),
    ("dot pads y with -0.0 instead of +0.0",
     "    float yv = e < e1 ? load_f(rk->y, rk->dtype, e) : 0.0f;",
     "    float yv = e < e1 ? load_f(rk->y, rk->dtype, e) : -0.0f;"),
    ("Dot2 correction added in another order",
     "      a->c = a->c + (pe + q);", "      a->c = (a->c + pe) + q;"),
    ("float sums pad with +0.0 instead of -0.0",
     "  float xv = e < e1 ? load_f(rk->x, rk->dtype, e) : -0.0f;",
     "  float xv = e < e1 ? load_f(rk->x, rk->dtype, e) : 0.0f;"),
    ("TwoSum tree combines the compensations in another order",
     "    r.c = (a.c + b.c) + e;", "    r.c = a.c + (b.c + e);"),
    ("shfl_up keeps its own value one lane too far",
     "  case SH_UP: return (l - b >= arg) ? l - arg : l;", "  case SH_UP: return (l - b > arg) ? l - arg : l;"),
    ("compaction keeps zeros",
     "(((const int32_t *)ck->x)[e] > 0);", "(((const int32_t *)ck->x)[e] >= 0);"),
    ("bitonic comparator direction flipped",
     "        key[l] = (lower == asc) ? mn : mx;", "        key[l] = (lower != asc) ? mn : mx;"),
    ("key-value insertion moves past equal keys (not stable)",
     "    while (j > 0 && k[j - 1] > kk) {", "    while (j > 0 && k[j - 1] >= kk) {"),
    ("row scan adds the shifted value one lane late",
     "      if ((l & 15) >= d) r[l] = sadd(isf, r[l], t[l]);", "      if ((l & 15) > d) r[l] = sadd(isf, r[l], t[l]);"),
    ("masked operations take the density bound inclusively",
     "  for (int l = 0; l < 32; l++) pr[l] = ((uint32_t)x[l] & 1023u) < (uint32_t)c->D;\n"
     "  for (int l = 0; l < 32; l++) xch_put(&X, l, (uint64_t)pr[l]);",
     "  for (int l = 0; l < 32; l++) pr[l] = ((uint32_t)x[l] & 1023u) <= (uint32_t)c->D;\n"
     "  for (int l = 0; l < 32; l++) xch_put(&X, l, (uint64_t)pr[l]);"),
    ("match_any leaves the calling lane out of its own set",
     "    if (((mask >> i) & 1u) && x->v[i] == x->v[l]) r |= 1u << i;",
     "    if (((mask >> i) & 1u) && i != l && x->v[i] == x->v[l]) r |= 1u << i;"),
    ("integral image rows scanned exclusively",
     "    s += c->img[y * c->W + x];\n    c->sat[y * c->W + x] = s;",
     "    c->sat[y * c->W + x] = s;\n    s += c->img[y * c->W + x];"),
    ("conjugate gradient beta as the inverse ratio",
     "    g.coef = k == 0 ? 0.0f : (float)(rr / rr_prev);", "    g.coef = k == 0 ? 0.0f : (float)(rr_prev / rr);"),
    ("conjugate gradient alpha as the inverse ratio",
     "    g.coef = (float)(rr / pq);", "    g.coef = (float)(pq / rr);"),
    ("segmented float scan carried in FP32",
     "      if (isf) ((float *)c->y)[e0 + o] = (float)(fcarry + (double)q[o].f);",
     "      if (isf) ((float *)c->y)[e0 + o] = (float)fcarry + q[o].f;"),
    ("segmented compaction written from the start of out, not the segment's offset",
     "    void *dst = isf ? (void *)((float *)c->outc + a + kept) : (void *)((int32_t *)c->outc + a + kept);",
     "    void *dst = isf ? (void *)((float *)c->outc + kept) : (void *)((int32_t *)c->outc + kept);"),
    ("segmented float totals rounded to FP32 per chunk",
     "    if (isf) ftot = ftot + (double)P.s;", "    if (isf) ftot = (float)(ftot + (double)P.s);"),
]


def run_pins(tmp_path, source):
    """Builds `source` as the oracle and runs the pin suites against it;
    returns the subprocess result."""
    from oracle import build as ob

    c = tmp_path / "coxo.c"
    c.write_text(source)
    lib = tmp_path / "libcoxo.so"
    subprocess.run(["gcc", *ob.CFLAGS, str(c), "-o", str(lib), "-lm"], check=True)
    env = dict(os.environ, COXO_LIB=str(lib))
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                           *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_unmutated_copy_passes(tmp_path):
    """The control: the same harness on an unchanged copy passes every pin."""
    r = run_pins(tmp_path, open(SRC).read())
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("what,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_a_pin_catches(tmp_path, what, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "the mutation site moved: " + old
    r = run_pins(tmp_path, src.replace(old, new))
    assert r.returncode == 1, f"no pin caught: {what}\n{r.stdout[-2000:]}"  # 1: tests failed (not an error)
