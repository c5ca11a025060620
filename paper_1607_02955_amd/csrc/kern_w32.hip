// Kernel instantiations for block width 32.
#include "kern_impl.hpp"
CFC_DEFINE_TABLES(32)
