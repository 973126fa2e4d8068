"""Helpers shared by the GPU tests: tensor <-> numpy word views and inputs."""
import numpy as np
import torch

import synth


def say(msg: str) -> None:
    print(msg, flush=True)


def dev():
    return torch.device("cuda:0")


def u32(t) -> np.ndarray:
    """Device int32/float32 tensor -> host uint32 words."""
    a = t.detach().cpu().contiguous().numpy()
    return a.view(np.uint32)


def states_t(arr: np.ndarray):
    arr = np.ascontiguousarray(arr, np.uint32).reshape(-1, 98)
    return torch.from_numpy(arr.view(np.int32).copy()).to(dev())


def jumps_t(Js):
    lo, hi = synth.int_to_u128(Js)
    return limbs_t(lo, hi)


def limbs_t(lo, hi):
    arr = np.stack([np.asarray(lo, np.uint64), np.asarray(hi, np.uint64)], 1)
    return torch.from_numpy(np.ascontiguousarray(arr).view(np.int64).copy()).to(dev())


def seeds_t(seeds):
    return torch.from_numpy(np.asarray(seeds, np.int32).copy()).to(dev())


def f32_words(k: np.ndarray) -> np.ndarray:
    """The float32 bit patterns of k * 2^-24 (exact), computed in float64."""
    return (k.astype(np.float64) * 2.0 ** -24).astype(np.float32).view(np.uint32)
