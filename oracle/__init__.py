"""FP64 CPU oracle of the butterfly-interaction particle filter.

TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. It shares no code with
the device path (``paper_1812_01502_amd``); the two meet only in the seeded
input generators of ``workloads``.

Modules:
  philox     Philox4x32-10 and the filter's random-number stream definition
  plan       radix/mixed-radix stage plan, butterfly groups, the paper's A_s
  models     log g, prior sampler and Markov kernel of the LG and SV models
  butterfly  the filter, one rotating butterfly stage per step
  bpf        the plain bootstrap filter (Algorithms 1 and 2), written apart
  augmented  full S-stage augmented resampling (Algorithm 3) and its exact law
  island     the island filter (AIRPF, Algorithms 4-7)
  adaptive   ESS-gated stages with a rotating start (Sections 1.2 and 6.4)
  kalman     Kalman filter (closed form for LG models)
  gridfilter point-mass filter for the SV model
"""
from . import adaptive, augmented, bpf, butterfly, gridfilter, island, kalman, models, philox, plan  # noqa: F401
from .butterfly import MULTINOMIAL, SYSTEMATIC, ButterflyOracle, State  # noqa: F401
from .island import IslandOracle  # noqa: F401
