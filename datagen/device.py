"""Device-side generation of the same synthetic inputs (libdatagen.so).

Keys and int64 values are bit-identical to the numpy generators in this
package; float64 normals use a counter-based Box-Muller transform instead of
numpy's PCG64 (tests that need them on the host copy them back)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import KEY_SALT, stream, substream_seed, zipf_cdf_table

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdatagen.so")
_lib = None


def build() -> str:
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           os.path.join(HERE, "gen.hip"), "-o", tmp])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdatagen.so is not built")
        # torch's HIP runtime must be the one the library binds to: loaded
        # first, it satisfies the library's libamdhip64 dependency; loaded
        # after, a second runtime would come up without the GPU
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        U, P = ctypes.c_uint64, ctypes.c_void_p
        L.dg_uniform_keys.argtypes = [U, U, U, U, U, P, P]
        L.dg_zipf_keys.argtypes = [U, U, U, P, U, U, P, P]
        L.dg_uniform_i64.argtypes = [U, U, U, ctypes.c_int64, U, P, P]
        L.dg_normal_f64.argtypes = [U, U, U, P, P]
        L.dg_zipf_approx_keys.argtypes = [U, U, U, U, ctypes.c_double, U, P, P]
        L.dg_uniform_ranks.argtypes = [U, U, U, U, P, P]
        L.dg_segment_b.argtypes = [U, U, U, U, P, P, P]
        _lib = L
    return _lib


def _st():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ck(rc):
    if rc != 0:
        raise RuntimeError("datagen kernel launch failed (%d)" % rc)


def keys(seed: int, n: int, d: int, s: float = 0.0, table_dev=None, start: int = 0, out=None):
    """uint64 keys (as an int64 tensor) over a d-value domain, uniform or Zipf s."""
    import torch
    L = _load()
    out = torch.empty(n, dtype=torch.int64, device="cuda") if out is None else out
    if s == 0:
        _ck(L.dg_uniform_keys(seed, start, n, d, int(KEY_SALT), out.data_ptr(), _st()))
    else:
        if table_dev is None:
            table_dev = torch.from_numpy(zipf_cdf_table(d, s).view(np.int64)).cuda()
        _ck(L.dg_zipf_keys(seed, start, n, table_dev.data_ptr(), d, int(KEY_SALT), out.data_ptr(), _st()))
    return out


def zipf_approx_keys(seed: int, n: int, d: int, s: float, start: int = 0, out=None):
    """Keys over a d-value domain with approximately Zipf(s) ranks (continuous
    inversion; no table), for domains too large for an exact CDF table."""
    import torch
    out = torch.empty(n, dtype=torch.int64, device="cuda") if out is None else out
    _ck(_load().dg_zipf_approx_keys(seed, start, n, d, float(s), int(KEY_SALT), out.data_ptr(), _st()))
    return out


def uniform_ranks(seed: int, n: int, d: int, start: int = 0, out=None):
    """int64 ranks uniform over [0, d) (datagen.uniform_ranks on the device)."""
    import torch
    out = torch.empty(n, dtype=torch.int64, device="cuda") if out is None else out
    _ck(_load().dg_uniform_ranks(seed, start, n, d, out.data_ptr(), _st()))
    return out


def uniform_i64(seed: int, n: int, lo: int = -1_000_000, hi: int = 1_000_000, start: int = 0, out=None):
    import torch
    out = torch.empty(n, dtype=torch.int64, device="cuda") if out is None else out
    _ck(_load().dg_uniform_i64(seed, start, n, lo, hi - lo + 1, out.data_ptr(), _st()))
    return out


def normal_f64(seed: int, n: int, start: int = 0, out=None):
    import torch
    out = torch.empty(n, dtype=torch.float64, device="cuda") if out is None else out
    _ck(_load().dg_normal_f64(seed, start, n, out.data_ptr(), _st()))
    return out


def plain_input(seed: int, n: int, d: int, s: float = 0.0, with_f64: bool = False, table_dev=None):
    """Device twin of datagen.plain_input (keys and int64 values bit-identical)."""
    k = keys(substream_seed(seed, 1), n, d, s, table_dev=table_dev)
    v = uniform_i64(substream_seed(seed, 2), n)
    f = normal_f64(substream_seed(seed, 3), n) if with_f64 else None
    return k, v, f


def segmented_input(seed: int, n: int, n_a: int = 1000, b_per_a: int = 100_000):
    """Device twin of datagen.segmented_input (all three columns bit-identical).
    The segment of each row is drawn on the device and sorted there."""
    import torch
    L = _load()
    cand = (stream(substream_seed(seed, 10), 0, 4 * n_a) >> np.uint64(32)).astype(np.uint32).view(np.int32)
    _, first = np.unique(cand, return_index=True)
    a_vals = np.sort(cand[np.sort(first)[:n_a]])
    n_a = a_vals.shape[0]
    seg = torch.empty(n, dtype=torch.int64, device="cuda")
    _ck(L.dg_uniform_ranks(substream_seed(seed, 11), 0, n, n_a, seg.data_ptr(), _st()))
    seg = torch.sort(seg).values
    a = torch.from_numpy(a_vals).cuda()[seg]
    b = torch.empty(n, dtype=torch.int32, device="cuda")
    _ck(L.dg_segment_b(substream_seed(seed, 12), n, b_per_a, substream_seed(seed, 13), seg.data_ptr(),
                       b.data_ptr(), _st()))
    del seg
    v = uniform_i64(substream_seed(seed, 14), n)
    return a, b, v
