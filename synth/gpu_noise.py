"""Device-side image noise for data sets whose images are regenerated batch
by batch (noise.hip, built into libsynth_noise.so next to this file).

The noise of a pixel depends only on (seed, image index, pixel), so a
regenerated image always carries the same noise.  Input synthesis only:
nothing of the method runs here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "noise.hip")
LIB = os.path.join(HERE, "libsynth_noise.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
TAG = 0x4E4F4953  # the stream tag in the generator's counter

_lib = None


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + [SOURCE, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError("libsynth_noise.so is not built; run `python -c 'import synth.gpu_noise as n; n.build()'`")
        L = ctypes.CDLL(LIB)
        L.synth_add_disk_noise.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p]
        L.synth_add_disk_noise.restype = ctypes.c_int
        _lib = L
    return _lib


def noise_seed(seed: int, stream: int) -> int:
    """The generator's 64-bit key for a data set's seed and sub-stream."""
    return ((int(seed) & 0xFFFFFFFFFFFFFF) << 8) | (int(stream) & 0xFF)


def add_disk_noise(x, idx, k2max: int, sigma2: float, key: int):
    """x += complex Gaussian noise of variance sigma2 on the disk
    kx^2 + ky^2 <= k2max of every image; x: complex64 [n, M, M] on the GPU
    (contiguous), idx: int64 [n] on the GPU, the data-set index of each
    image; key from noise_seed.  Runs on torch's current stream."""
    import torch
    if x.dtype != torch.complex64 or not x.is_cuda or not x.is_contiguous() or x.dim() != 3 or x.shape[1] != x.shape[2]:
        raise ValueError("x must be a contiguous complex64 [n, M, M] GPU tensor")
    if idx.dtype != torch.int64 or idx.device != x.device or idx.numel() != x.shape[0]:
        raise ValueError("idx must be an int64 tensor of n indices on the same device")
    idx = idx.contiguous()
    stream = torch.cuda.current_stream(x.device).cuda_stream
    rc = lib().synth_add_disk_noise(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(idx.data_ptr()), x.shape[0],
                                    x.shape[1], int(k2max), float(sigma2), int(key) & 0xFFFFFFFFFFFFFFFF,
                                    ctypes.c_void_p(stream))
    if rc != 0:
        raise RuntimeError("synth_add_disk_noise failed with code %d" % rc)
    return x
