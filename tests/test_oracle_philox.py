"""Pins of the oracle's Philox4x32-10 (random numbers are unspecified in the
paper; the counter-based generator is the reading both sides implement)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[:4], v[4:6], v[6:10]))
    return rows


def test_known_answer_vectors(orc):
    for ctr, key, out in _kat():
        assert list(orc.philox4x32_10(ctr, key)) == out


_ROCRAND_SRC = r"""
#include <cstdio>
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
int main(){
  unsigned c0,c1,c2,c3,k0,k1;
  while(scanf("%x %x %x %x %x %x",&c0,&c1,&c2,&c3,&k0,&k1)==6){
    rocrand_state_philox4x32_10 st;
    unsigned long long seed=((unsigned long long)k1<<32)|k0;
    unsigned long long sub=((unsigned long long)c3<<32)|c2;
    unsigned long long off=4ull*(((unsigned long long)c1<<32)|c0);
    rocrand_init(seed,sub,off,&st);
    uint4 r=rocrand4(&st);
    printf("%08x %08x %08x %08x\n",r.x,r.y,r.z,r.w);
  }
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_matches_rocrand_host_implementation(orc, tmp_path):
    """rocRAND's own Philox4x32-10 (host build of its header) on random
    counters: rocrand_init(seed=key, subsequence=ctr[2:4], offset=4*ctr[0:2])
    makes the first rocrand4() the block at exactly that counter."""
    src = tmp_path / "rr.cpp"
    src.write_text(_ROCRAND_SRC)
    exe = tmp_path / "rr"
    subprocess.run(["hipcc", "-x", "c++", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                    "-O1", "-o", str(exe), str(src)], check=True, capture_output=True)
    rng = np.random.default_rng(7)
    n = 200
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64)
    ctr[:, 1] &= (1 << 30) - 1  # keep 4 * (ctr1:ctr0) inside 64 bits
    key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64)
    lines = "\n".join(" ".join("%08x" % int(v) for v in list(c) + list(k)) for c, k in zip(ctr, key))
    out = subprocess.run([str(exe)], input=lines, capture_output=True, text=True, check=True).stdout
    got = [[int(t, 16) for t in l.split()] for l in out.strip().splitlines()]
    assert len(got) == n
    for c, k, g in zip(ctr, key, got):
        assert list(orc.philox4x32_10(c.astype(np.uint32), k.astype(np.uint32))) == g


def test_output_bits_are_balanced(orc):
    """Crude sanity: each output bit is set about half the time."""
    bits = np.zeros(128)
    n = 4000
    for i in range(n):
        w = orc.philox4x32_10([i, 3, 5, 0], [11, 13])
        for j in range(4):
            bits[32 * j:32 * j + 32] += (int(w[j]) >> np.arange(32)) & 1
    frac = bits / n
    assert np.all(np.abs(frac - 0.5) < 5 * 0.5 / np.sqrt(n))
