"""Plant plausible mistakes in copies of the oracle and check that the pins
catch every one of them.  Each mutant is compiled from a modified copy of
oracle/oracle.c and exercised in a child process (a mutant may crash, which
also counts as caught).  Nothing here touches the GPU."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, text in oracle.c, replacement)
MUTANTS = [
    ("counting sort places forward (unstable)",
     "for (uint64_t j = n; j-- > 0;) {", "for (uint64_t j = 0; j < n; j++) {"),
    ("prefix sum drops a term",
     "for (uint64_t i = 1; i < k; i++) C[i] += C[i - 1];", "for (uint64_t i = 2; i < k; i++) C[i] += C[i - 1];"),
    ("digit mask off by one",
     "const uint64_t mask = k - 1;", "const uint64_t mask = k >> 1;"),
    ("pass count rounds down",
     "d = (key_bits + (unsigned)r - 1) / (unsigned)r;", "d = key_bits / (unsigned)r;"),
    ("insertion sort with >= (unstable)",
     "while (i >= 0 && a[i] > key) {", "while (i >= 0 && a[i] >= key) {"),
    ("merge takes right run on ties (unstable)",
     "if (src[i] <= src[j]) {", "if (src[i] < src[j]) {"),
    ("bucket range without the +1",
     "u128 range = (u128)mx - (u128)mn + 1;", "u128 range = (u128)mx - (u128)mn + 2;"),
    ("bucket map in 64-bit arithmetic",
     "u128 num = (u128)(k - mn) * (u128)B;", "u128 num = (u128)((k - mn) * B);"),
    ("buckets filled last-to-first",
     "for (uint64_t i = 0; i < n; i++) {\n        uint64_t b = BUCKET(A[i]);",
     "for (uint64_t i = n; i-- > 0;) {\n        uint64_t b = BUCKET(A[i]);"),
    ("declared range ignored",
     "if (key_bound) {", "if (0) {"),
    ("min taken as the first key",
     "if (A[i] < mn) mn = A[i];", "if (0) mn = A[i];"),
    ("payload not moved in the digit sort",
     "if (VA) VB[C[dg]] = VA[j];", "if (VA) VB[C[dg]] = VA[C[dg]];"),
    ("signed keys compared as unsigned",
     "return sa < sb;", "return a < b;"),
    ("float sign orders positives first",
     "if (neg_a != neg_b) return neg_a > neg_b;", "if (neg_a != neg_b) return neg_a < neg_b;"),
    ("negative floats by ascending magnitude",
     "if (neg_a) return ma > mb;", "if (neg_a) return ma < mb;"),
    ("sign bit of 32-bit keys taken from bit 63",
     "const unsigned top = 8u * (unsigned)key_bytes - 1u;", "const unsigned top = 63u;"),
    ("bucket starts exported one bucket late",
     "if (offsets) memcpy(offsets, off, (nbuckets + 1) * sizeof(uint64_t));",
     "if (offsets) { memcpy(offsets, off + 1, nbuckets * sizeof(uint64_t)); offsets[nbuckets] = n; }"),
    ("ordered merge takes right run on ties",
     "(j < hi && key_before(src[j], src[i], key_bytes, order))",
     "(j < hi && !key_before(src[i], src[j], key_bytes, order))"),
]

CHECK = textwrap.dedent(r'''
    import sys, itertools
    import numpy as np
    sys.path.insert(0, ROOT)
    import oracle
    oracle._lib = oracle._load(LIB)
    rng = np.random.default_rng(7)
    def ref(k, v):
        o = np.argsort(k, kind="stable"); return k[o], v[o]
    def same(res, k, v):
        ek, ev = ref(k, v)
        return np.array_equal(res.keys, ek) and np.array_equal(res.vals, ev)
    ok = True
    # brute force: every sequence of length <= 5 over {0..3}
    for n in range(6):
        for seq in itertools.product(range(4), repeat=n):
            k = np.array(seq, dtype=np.uint32); v = np.arange(n, dtype=np.uint32)
            ok &= same(oracle.radix_lsd(k, v, r=2), k, v)
            ok &= same(oracle.bucket(k, v, num_buckets=3, cutoff=4), k, v)
    # random u32/u64 against the library stable sort, several widths
    for dt, hi in ((np.uint32, 1 << 32), (np.uint64, 1 << 64)):
        k = rng.integers(0, min(hi, 1 << 63), 3000, dtype=np.uint64).astype(dt)
        if dt == np.uint64: k = k * np.uint64(2) + rng.integers(0, 2, 3000, dtype=np.uint64)
        k[::7] = k[3]
        v = np.arange(3000, dtype=np.uint32)
        for r in (8, 11):
            ok &= same(oracle.radix_lsd(k, v, r=r), k, v)
        for B, cut in ((1024, 32), (16, 8), (65536, 32)):
            ok &= same(oracle.bucket(k, v, num_buckets=B, cutoff=cut), k, v)
    # exact bucket map at the 64-bit range and its boundaries
    mx = (1 << 64) - 1
    for kk in (0, 1 << 63, mx):
        ok &= oracle.bucket_index(kk, 0, mx, 1024) == (kk * 1024) >> 64
    for (mn, mxx, B) in ((0, 2**32 - 1, 1024), (17, 1040, 7), (2**40, 2**41, 1000)):
        R = mxx - mn + 1
        for j in range(1, B):
            f = mn + -(-j * R // B)
            ok &= oracle.bucket_index(f, mn, mxx, B) == (f - mn) * B // R
    # bucket intermediates: scatter is the stable partition by bucket
    k = rng.integers(0, 1 << 32, 2000, dtype=np.uint64).astype(np.uint32)
    v = np.arange(2000, dtype=np.uint32)
    res = oracle.bucket(k, v, num_buckets=64, cutoff=8, want_intermediates=True)
    mn, mxx = int(k.min()), int(k.max())
    b = np.array([(int(x) - mn) * 64 // (mxx - mn + 1) for x in k])
    ok &= (res.kmin, res.kmax) == (mn, mxx)
    ok &= np.array_equal(res.scat_keys, k[np.argsort(b, kind="stable")])
    # declared range [0, M] with B = n: the map floor(n*k/(M+1))
    kk = rng.integers(0, 10**6 + 1, 3000, dtype=np.uint64).astype(np.uint32)
    res = oracle.bucket(kk, num_buckets=3000, key_bound=10**6, want_intermediates=True)
    want = np.bincount([(3000 * int(x)) // (10**6 + 1) for x in kk], minlength=3000)
    ok &= np.array_equal(res.counts.astype(np.int64), want)
    # bucket starts: the first position of the scatter whose bucket is at
    # least b, across wide gaps of empty buckets
    kk = rng.choice(np.array([0, 7, 1 << 20, (1 << 31) + 5, (1 << 32) - 1], dtype=np.uint64), 500).astype(np.uint32)
    res = oracle.bucket(kk, num_buckets=4096, want_intermediates=True)
    bs = np.array([(int(x) * 4096) // (1 << 32) for x in res.scat_keys])
    ok &= np.array_equal(res.offsets.astype(np.int64), np.searchsorted(bs, np.arange(4097), side="left"))
    # signed keys against the library sort; IEEE keys on a totalOrder ladder
    for dt in (np.int32, np.int64):
        info = np.iinfo(dt)
        k = rng.integers(info.min, info.max, 3000, dtype=dt, endpoint=True)
        k[::7] = k[3]
        v = np.arange(3000, dtype=np.uint32)
        rk, rv = oracle.sort_ordered(k, v)
        ek, ev = ref(k, v)
        ok &= np.array_equal(rk, ek) and np.array_equal(rv, ev)
    for fdt, ut, lad in ((np.float32, np.uint32, [0xFFC00000, 0xFF800000, 0xBF800000, 0x80000000,
                                                  0x00000000, 0x3F800000, 0x7F800000, 0x7FC00000]),
                         (np.float64, np.uint64, [0xFFF8000000000000, 0xFFF0000000000000,
                                                  0xBFF0000000000000, 0x8000000000000000, 0,
                                                  0x3FF0000000000000, 0x7FF0000000000000,
                                                  0x7FF8000000000000])):
        lad = np.array(lad, dtype=ut)
        idx = np.repeat(np.arange(lad.size), 3)
        rng.shuffle(idx)
        v = np.arange(idx.size, dtype=np.uint32)
        rk, rv = oracle.sort_ordered(lad[idx].view(fdt), v)
        o = np.argsort(idx, kind="stable")
        ok &= np.array_equal(rk.view(ut), lad[idx[o]]) and np.array_equal(rv, v[o])
    sys.exit(0 if ok else 3)
''')


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique/found: {name}"
    mutant = tmp_path / "oracle_mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", str(mutant), "-o", str(lib)], check=True)
    prog = f"ROOT = {ROOT!r}\nLIB = {str(lib)!r}\n" + CHECK
    rc = subprocess.run([sys.executable, "-c", prog], timeout=300).returncode
    assert rc != 0, f"pins did not catch mutant: {name}"


def test_unmutated_oracle_passes_the_same_checks(tmp_path):
    lib = tmp_path / "liboracle_clean.so"
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", SRC, "-o", str(lib)], check=True)
    prog = f"ROOT = {ROOT!r}\nLIB = {str(lib)!r}\n" + CHECK
    assert subprocess.run([sys.executable, "-c", prog], timeout=300).returncode == 0
