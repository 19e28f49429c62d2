// Device code instantiated for N = 8.
#include "engine.hpp"

namespace psdns {
Ops ops_n8(int precision) {
  return precision == 32 ? Engine<8, float>::ops() : Engine<8, double>::ops();
}
}  // namespace psdns
