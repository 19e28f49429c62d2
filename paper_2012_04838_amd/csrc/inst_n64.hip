// Device code instantiated for N = 64.
#include "engine.hpp"

namespace psdns {
Ops ops_n64(int precision) {
  return precision == 32 ? Engine<64, float>::ops() : Engine<64, double>::ops();
}
}  // namespace psdns
