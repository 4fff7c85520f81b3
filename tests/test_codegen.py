"""Code-generation checks on the gfx950 build (CPU: hipcc cross-compiles).

The persistent SpGEMM kernels pull rows from a global counter.  Written as an
endless loop with the fetch at its top, the compiler routed threads other
than 0 from the end of the body past the fetch, and the generated code kept
those lanes in an inner loop over one row that they never left.  These tests
compile the kernels to assembly and check that every loop reading the
broadcast row index also contains the counter atomic; a small kernel in the
old shape checks that the check itself sees the fault."""

import os
import subprocess

import pytest

from asm_loops import check
from paper_1512_00066_amd import build as B

pytestmark = pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")

OLD_SHAPE = r"""
#include <hip/hip_runtime.h>
__device__ __forceinline__ long long fetch(unsigned long long *ctr) {
  __shared__ long long r;
  if (threadIdx.x == 0) r = (long long)atomicAdd(ctr, 1ull);
  __syncthreads();
  const long long v = r;
  __syncthreads();
  return v;
}
__global__ void __launch_bounds__(64) rows_old(unsigned long long *ctr, long long count, const int *in,
                                               long long *out) {
  __shared__ long long part[2];
  for (;;) {
    const long long r = fetch(ctr);
    if (r >= count) break;
    long long s = in[r * 64 + threadIdx.x];
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if (threadIdx.x == 0) part[0] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[r] = part[0];
  }
}
"""


def _asm_of(src_text, tmp_path, name):
    src = tmp_path / (name + ".hip")
    src.write_text(src_text)
    out = tmp_path / (name + ".s")
    flags = [f for f in B.FLAGS if f != "-fPIC"]
    r = subprocess.run([B.HIPCC, *flags, "-x", "hip", "--cuda-device-only", "-S", str(src), "-o", str(out)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out.read_text()


def test_checker_flags_old_loop_shape(tmp_path):
    kernels, bad = check(_asm_of(OLD_SHAPE, tmp_path, "old_shape"))
    assert kernels == 1
    assert bad, "a loop over the row slot without the counter atomic should be reported"


def test_spgemm_persistent_loops_contain_their_fetch(tmp_path):
    out = B.device_asm("spgemm.hip", str(tmp_path / "spgemm.s"))
    kernels, bad = check(open(out).read())
    # symbolic (4 hash + bitmap) and numeric (hash, dense) kernels of every semiring
    assert kernels >= 40
    assert not bad, bad[:5]
