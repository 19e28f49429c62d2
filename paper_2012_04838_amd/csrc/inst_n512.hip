// Device code instantiated for N = 512, FP32 (the FP64 kernels are in their own
// translation unit so that the two compile in parallel).
#include "engine.hpp"

namespace psdns {
Ops ops_n512_f64();
Ops ops_n512(int precision) { return precision == 32 ? Engine<512, float>::ops() : ops_n512_f64(); }
}  // namespace psdns
