// Learned initial guess (internal header).
#pragma once

#include "bim.h"
