// Device code instantiated for N = 1024.
#include "engine.hpp"

namespace psdns {
Ops ops_n1024(int precision) {
  return precision == 32 ? Engine<1024, float>::ops() : Engine<1024, double>::ops();
}
}  // namespace psdns
