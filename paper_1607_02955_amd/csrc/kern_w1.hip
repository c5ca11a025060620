// Kernel instantiations for block width 1.
#include "kern_impl.hpp"
CFC_DEFINE_TABLES(1)
