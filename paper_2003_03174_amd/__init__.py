"""MI355X-native TRD track-to-tracklet matching (Kalman filter over six layers).

The compute path lives in the HIP/C library under csrc/ behind the C ABI in
include/trd.h; `binding` is its thin Python marshalling layer and `synth` the
seeded workload generator.
"""
