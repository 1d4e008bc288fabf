"""Algorithmic operation counts of the Independent-algorithm hot path and the
MI355X VALU peak they are priced against.

The hot loop is integer hashing plus f64 waiting-time arithmetic with small
table gathers; nothing is a dense contraction, so the bound is the vector ALU.
Counts are per operation of the method as specified (one 32x32->64 product =
2 lane-ops, one 3-input xor = 2, one f64 fma = 1, one f64 divide = 1):

* Philox4x32-10 block: 10 rounds x (2 products x 2 + 2 three-input xors x 2
  + 2 key increments) = 100 lane-ops.
* Exponential draw: 53-bit uniform (4), exponent/mantissa split on the integer
  (15), log series (19 f64 ops: subtract, add, divide, square, 9 fma, multiply,
  doubling, 3 fma, convert), negate/scale/accumulate/two compares (5) = 43.
* Event bookkeeping besides its Philox blocks: speciation compare (3), two
  64x32 index products (14), alias gather address and coin (6), offset decode
  and torus wrap (12), target, deme index and packed location (5) = 40.

The peak is the VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz =
39.3e12 lane-ops/s (the same rate at which f64 FMAs give 78.6 TFLOP/s).
"""
OPS_PER_PHILOX = 100
OPS_PER_DRAW = 43
OPS_PER_EVENT = 40

N_CU = 256
LANES_PER_CU_CLK = 64
CLOCK_HZ = 2.4e9
PEAK_LANE_OPS = N_CU * LANES_PER_CU_CLK * CLOCK_HZ  # 3.93e13 lane-ops/s


# Per-deme dispersal (heterogeneous habitat): per dispersal one 16-byte alias entry (which also
# carries both candidate targets' capacities) and the deme's two row pointers (8 B) are gathered
# from HBM-resident tables.
BYTES_PER_DISPERSAL_PER_DEME = 24


def algorithmic_ops(philox_calls: int, exp_draws: int, events: int) -> float:
    return OPS_PER_PHILOX * philox_calls + OPS_PER_DRAW * exp_draws + OPS_PER_EVENT * events
