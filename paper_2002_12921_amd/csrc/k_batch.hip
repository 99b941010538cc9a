// placeholder, replaced by the batched persistent kernel
#include "device_common.hpp"
