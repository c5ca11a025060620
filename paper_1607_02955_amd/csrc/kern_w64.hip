// Kernel instantiations for block width 64.
#include "kern_impl.hpp"
CFC_DEFINE_TABLES(64)
