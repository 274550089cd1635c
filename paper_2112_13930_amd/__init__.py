"""MI355X-native fused lattice-kinetic MHD step with Shercliff wall closures.

The compute path is the HIP library ``liblks_mhd.so`` (C ABI in
``include/lks_mhd.h``); this package only marshals arguments and owns device
memory through PyTorch.

  Channel  one channel (``channel.py``)
  Batch    many channels advanced together (``batch.py``)
  Server   continuous-batching solve service (``serve.py``)
"""
from ._lib import (BCS, LKS_BC_LINK, LKS_BC_MOMENT, LKS_EDEVICE, LKS_EINVAL,  # noqa: F401
                   LKS_ENOMEM, LKS_ENOTCONV, LKS_EUNSTABLE, LKS_FP16_STORE, LKS_FP16_STORE_F64, LKS_FP32,
                   LKS_FP64, LKS_OK, PRECISIONS, LksError, LksParams, derive, lib,
                   make_params)


def __getattr__(name):
    if name == "Channel":
        from .channel import Channel
        return Channel
    if name == "Batch":
        from .batch import Batch
        return Batch
    if name == "Server":
        from .serve import Server
        return Server
    raise AttributeError(name)
