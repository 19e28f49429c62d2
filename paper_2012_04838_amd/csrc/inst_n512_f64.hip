// Device code instantiated for N = 512, FP64.
#include "engine.hpp"

namespace psdns {
Ops ops_n512_f64() { return Engine<512, double>::ops(); }
}  // namespace psdns
