// Device code instantiated for N = 16.
#include "engine.hpp"

namespace psdns {
Ops ops_n16(int precision) {
  return precision == 32 ? Engine<16, float>::ops() : Engine<16, double>::ops();
}
}  // namespace psdns
