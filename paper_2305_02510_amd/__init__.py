"""MI355X-native simulator of homogeneous LIF networks with synaptic delays
(the matrix-form mode of SuperNeuro, Date et al., ICONS'23, §2.1).

The simulation runs in the HIP library ``libsnmi.so`` (C ABI in
``include/superneuro_mi.h``); ``Network`` marshals arguments to it, with
PyTorch providing device memory and the stream.
"""
from .network import Batch, Network, pack_bits, unpack_bits  # noqa: F401
