// Device code instantiated for N = 512.
#include "engine.hpp"

namespace psdns {
Ops ops_n512(int precision) {
  return precision == 32 ? Engine<512, float>::ops() : Engine<512, double>::ops();
}
}  // namespace psdns
