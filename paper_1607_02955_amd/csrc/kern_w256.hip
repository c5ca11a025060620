// Kernel instantiations for block width 256.
#include "kern_impl.hpp"
CFC_DEFINE_TABLES(256)
