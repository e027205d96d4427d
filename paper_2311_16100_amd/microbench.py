"""Throughput probes and single-entry-point timings, for profiling.

  python -m paper_2311_16100_amd.microbench lds      LDS atomic add rates (u32, u64, f32, f64)
  python -m paper_2311_16100_amd.microbench scatter  complex contributions to random LDS voxels,
                                                     per accumulator design
  python -m paper_2311_16100_amd.microbench valu     vector FMA issue rate
  python -m paper_2311_16100_amd.microbench learned_diag [--M 256]
                                                     the learned preconditioner's volume inference
  python -m paper_2311_16100_amd.microbench mlp_grad [--n 8192]
                                                     one training-gradient launch of the network

Rates are given per compute unit and per clock at the 2.4 GHz peak engine
clock and 256 compute units (the chip's published figures; a lower actual
clock makes the per-clock figures conservative).  The probes live in
libcsg_microbench.so, a library of their own; the entry-point timings call
libcryosgd.so through its binding like any user.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

CUS, CLOCK_HZ = 256, 2.4e9
HERE = os.path.dirname(os.path.abspath(__file__))
MB_LIB = os.path.join(HERE, "libcsg_microbench.so")


def _mb():
    if not os.path.exists(MB_LIB):
        raise RuntimeError("libcsg_microbench.so is not built; run `python paper_2311_16100_amd/build.py`")
    L = ctypes.CDLL(MB_LIB)
    L.csg_mb_lds_add.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.csg_mb_lds_add.restype = ctypes.c_float
    L.csg_mb_lds_scatter.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    L.csg_mb_lds_scatter.restype = ctypes.c_float
    L.csg_mb_valu_fma.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    L.csg_mb_valu_fma.restype = ctypes.c_float
    return L


def lds(blocks_per_cu=(1, 2, 4, 8), reps=4096, strides=(1,)):
    import torch
    L = _mb()
    out = []
    for kind, name in ((0, "u32"), (1, "u64"), (2, "f32"), (3, "f64")):
        for bpc in blocks_per_cu:
            for stride in strides:
                blocks = CUS * bpc
                buf = torch.zeros(blocks, dtype=torch.float64, device="cuda")
                r = reps if kind != 2 else max(64, reps // 16)  # float LDS adds are slow: fewer reps
                ms = L.csg_mb_lds_add(kind, ctypes.c_void_p(buf.data_ptr()), blocks, r, stride)
                if ms <= 0:
                    raise RuntimeError("probe failed")
                ops = blocks * 256 * r
                rate = ops / (ms * 1e-3)
                out.append({"type": name, "blocks_per_cu": bpc, "stride": stride, "reps": r, "ms": round(ms, 4),
                            "lane_ops_per_s": rate, "per_cu_per_clock": round(rate / (CUS * CLOCK_HZ), 3)})
    return out


SCATTER_DESIGNS = {0: "two ds_add_u64", 1: "one packed ds_add_u64", 2: "two ds_add_rtn_u32 + carry",
                   3: "two ds_add_u32 (no carry)", 4: "one packed ds_add_rtn_u64 + carry"}


def scatter(blocks_per_cu=(2, 4), reps=4096):
    """Complex contributions per clock per CU scattered to random LDS
    voxels, for each accumulator design of csg_mb_lds_scatter."""
    import torch
    L = _mb()
    out = []
    for design, name in SCATTER_DESIGNS.items():
        for bpc in blocks_per_cu:
            blocks = CUS * bpc
            buf = torch.zeros(blocks, dtype=torch.float64, device="cuda")
            ms = L.csg_mb_lds_scatter(design, ctypes.c_void_p(buf.data_ptr()), blocks, reps)
            if ms <= 0:
                raise RuntimeError("probe failed")
            n = blocks * 256 * reps
            rate = n / (ms * 1e-3)
            out.append({"design": name, "blocks_per_cu": bpc, "reps": reps, "ms": round(ms, 4),
                        "contributions_per_cu_per_clock": round(rate / (CUS * CLOCK_HZ), 3),
                        "lds_cycles_per_wave_contribution": round(64 * CUS * CLOCK_HZ / rate, 2)})
    return out


def valu(blocks_per_cu=(4, 8, 16), reps=20000):
    import torch
    L = _mb()
    out = []
    for bpc in blocks_per_cu:
        blocks = CUS * bpc
        buf = torch.zeros(blocks * 256, dtype=torch.float32, device="cuda")
        ms = L.csg_mb_valu_fma(ctypes.c_void_p(buf.data_ptr()), blocks, reps)
        lane_fma = blocks * 256 * reps * 8
        rate = lane_fma / (ms * 1e-3)
        out.append({"blocks_per_cu": bpc, "ms": round(ms, 4), "lane_fma_per_s": rate,
                    "wave_instr_per_cu_per_clock": round(rate / 64 / (CUS * CLOCK_HZ), 3),
                    "tflops": round(2 * rate / 1e12, 1)})
    return out


def _timed(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps


def learned_diag(M=256, reps=5, n_images=8192):
    """csg_learned_diag over the M^3 grid with features from n_images images
    of the high-resolution workload and a seeded random network."""
    import numpy as np
    import torch

    import synth
    from . import binding as B
    dev = torch.device("cuda:0")
    W = synth.WORKLOADS["hires_256"]
    g, o = B.Grid(M), B.Optics()
    rot = torch.from_numpy(synth.uniform_rotations(n_images, W.seed)).to(dev)
    df = torch.from_numpy(synth.defocus_values(n_images, *W.defocus_um, W.seed)).to(dev)
    acc = B.feature_sums(g, o, rot, df)
    ctf2, cover = acc.real.contiguous(), acc.imag.contiguous()
    rng = np.random.default_rng([7, synth.STREAM_MLP])
    params = torch.from_numpy((rng.standard_normal(B.mlp_param_count()) * 0.2).astype(np.float32)).to(dev)
    out = torch.empty((M, M, M), dtype=torch.float32, device=dev)
    ms = _timed(lambda: B.learned_diag(g, n_images, 1e-3, params, ctf2, cover, out=out), reps)
    reached = int((cover > 0).sum().item())
    return {"M": M, "voxels": M ** 3, "voxels_reached": reached, "ms": round(ms, 4), "reps": reps}


def mlp_grad(n=8192, reps=20):
    import numpy as np
    import torch

    import synth
    from . import binding as B
    dev = torch.device("cuda:0")
    rng = np.random.default_rng([8, synth.STREAM_MLP])
    params = torch.from_numpy((rng.standard_normal(B.mlp_param_count()) * 0.2).astype(np.float32)).to(dev)
    X = torch.from_numpy(rng.standard_normal((n, 3)).astype(np.float32)).to(dev)
    T = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to(dev)
    grad = torch.empty(B.mlp_param_count(), dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    ms = _timed(lambda: B.mlp_grad(params, X, T, grad=grad, loss=loss), reps)
    return {"n": n, "ms": round(ms, 4), "reps": reps}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("what", choices=["lds", "scatter", "valu", "learned_diag", "mlp_grad"])
    ap.add_argument("--M", type=int, default=256)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args(argv)
    if a.what == "lds":
        res = lds()
    elif a.what == "scatter":
        res = scatter()
    elif a.what == "valu":
        res = valu()
    elif a.what == "learned_diag":
        res = learned_diag(a.M, a.reps)
    else:
        res = mlp_grad(a.n, max(a.reps, 20))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    sys.exit(main())
