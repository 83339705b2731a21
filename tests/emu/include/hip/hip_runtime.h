#pragma once
#include "../../emu_shim.h"
