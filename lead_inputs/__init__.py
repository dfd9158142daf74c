"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark: finite groups, (A, B, C_A, C_B) code descriptions and channel
noise.  This package holds no decoding arithmetic; both decoders build the
code and decode on their own."""
from .groups import Group, cyclic, elementary_abelian2, dihedral, alternating5, psl2, by_name  # noqa: F401
from .codes import CodeSpec, sample_code, custom_code, standard, STANDARD  # noqa: F401
from .noise import (pack_bits, unpack_bits, words_for, bitflip_packed,  # noqa: F401
                    depolarizing_packed, uniform_p, channel_llr)
