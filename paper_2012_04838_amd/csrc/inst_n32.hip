// Device code instantiated for N = 32.
#include "engine.hpp"

namespace psdns {
Ops ops_n32(int precision) {
  return precision == 32 ? Engine<32, float>::ops() : Engine<32, double>::ops();
}
}  // namespace psdns
