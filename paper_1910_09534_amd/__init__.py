"""MI355X-native sliced state-vector engine (Schroedinger contraction of a
subcircuit slice's amplitude tensor with fused dense blocks, diagonal phase
folding, qubit-index permutes and a host-memory slice tier).

The HIP library is loaded lazily by `paper_1910_09534_amd.sv`; importing the
package itself touches no GPU and no native code.
"""
__version__ = "0.1.0"
