"""Helpers shared by the GPU parity tests."""
import numpy as np
import torch

DEV = "cuda:0"
NP = {"u32": np.uint32, "i32": np.int32, "f32": np.float32}

# sizes around every tile, wavefront and workgroup boundary of the kernels
BOUNDARY_SIZES = [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 15, 16, 17, 31, 32, 33, 63, 64, 65, 255, 256,
                  257, 511, 512, 513, 1023, 1024, 1025, 2047, 2049, 4095, 4096, 4097, 8191, 8192,
                  8193, 12289, 16383, 16384, 16385, 32769, 65535, 65536, 65537, 100003, 262145]


def say(msg):
    print(msg, flush=True)


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.cpu().numpy()


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def float_keys(n, seed):
    """Normal floats rounded to 1/8 (many ties, both zeros) plus +-inf and NaNs
    with assorted payloads."""
    rng = np.random.default_rng(seed)
    x = (np.round(rng.standard_normal(n) * 8) / 8).astype(np.float32)
    if n >= 16:
        idx = rng.choice(n, size=min(n, 12), replace=False)
        specials = np.array([0x7fc00000, 0xffc00000, 0x7f800001, 0xff812345, 0x7f800000,
                             0xff800000, 0x80000000, 0x00000000, 0x00000001, 0x80000001,
                             0x7f7fffff, 0xff7fffff], dtype=np.uint32).view(np.float32)
        x[idx] = specials[: idx.shape[0]]
    return x


def make_keys(n, dtype, seed, dist="random"):
    from paper_2503_05934_amd import workloads

    if dtype == "f32":
        return float_keys(n, seed)
    return workloads.keys(n, dist, dtype, seed)
