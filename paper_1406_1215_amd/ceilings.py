"""Binding of libclceil.so (include/clceil.h): the memory-system ceilings
the benchmark measures beside the generation kernel (random 8-byte gathers
from the weight array, plain 16-byte stores).  Argument marshalling only;
the kernels are in csrc/cl_ceilings.hip."""
from __future__ import annotations

import ctypes
import os

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libclceil.so")
THREADS = 256
_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, U64, U32, I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    L.clc_gather_uniform.argtypes = [P, U64, U64, U64, U32, P, P]
    L.clc_gather_uniform.restype = I
    L.clc_gather_list.argtypes = [P, U64, P, U64, U32, P, P]
    L.clc_gather_list.restype = I
    L.clc_store.argtypes = [P, U64, U32, P]
    L.clc_store.restype = I
    _lib = L
    return L


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(code, what):
    if code != 0:
        raise RuntimeError(f"{what} failed ({code})")


def out_buffer(blocks: int, device) -> torch.Tensor:
    return torch.empty(blocks * THREADS, dtype=torch.float64, device=device)


def gather_uniform(w: torch.Tensor, count: int, seed: int, blocks: int, out: torch.Tensor) -> None:
    assert w.dtype == torch.float64 and w.is_contiguous() and out.numel() >= blocks * THREADS
    _check(lib().clc_gather_uniform(w.data_ptr(), w.numel(), int(count), int(seed), int(blocks), out.data_ptr(),
                                    _stream()), "clc_gather_uniform")


def gather_list(w: torch.Tensor, idx: torch.Tensor, blocks: int, out: torch.Tensor) -> None:
    assert w.dtype == torch.float64 and idx.dtype == torch.int32 and idx.is_contiguous()
    assert out.numel() >= blocks * THREADS
    _check(lib().clc_gather_list(w.data_ptr(), w.numel(), idx.data_ptr(), idx.numel(), int(blocks), out.data_ptr(),
                                 _stream()), "clc_gather_list")


def store(buf: torch.Tensor, blocks: int) -> None:
    assert buf.is_contiguous()
    _check(lib().clc_store(buf.data_ptr(), buf.numel() * buf.element_size(), int(blocks), _stream()), "clc_store")
