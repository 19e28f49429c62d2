// Device code instantiated for N = 128.
#include "engine.hpp"

namespace psdns {
Ops ops_n128(int precision) {
  return precision == 32 ? Engine<128, float>::ops() : Engine<128, double>::ops();
}
}  // namespace psdns
