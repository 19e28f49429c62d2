// Device code instantiated for N = 256.
#include "engine.hpp"

namespace psdns {
Ops ops_n256(int precision) {
  return precision == 32 ? Engine<256, float>::ops() : Engine<256, double>::ops();
}
}  // namespace psdns
