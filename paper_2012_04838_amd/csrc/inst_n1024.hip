// Device code instantiated for N = 1024, FP32 (the FP64 kernels are in their own
// translation unit so that the two compile in parallel).
#include "engine.hpp"

namespace psdns {
Ops ops_n1024_f64();
Ops ops_n1024(int precision) { return precision == 32 ? Engine<1024, float>::ops() : ops_n1024_f64(); }
}  // namespace psdns
