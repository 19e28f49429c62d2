// Device code instantiated for N = 1024, FP64.
#include "engine.hpp"

namespace psdns {
Ops ops_n1024_f64() { return Engine<1024, double>::ops(); }
}  // namespace psdns
